"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Inputs are seeded synthetic images from ``synth``; expected values come from
the oracle only.  Tolerances: integer/index outputs bit-exact; G 1e-12 abs;
coefficients 1e-13 relative; one FP64 step (both sides starting from the
oracle's u^{resc;n-1}) 1e-10 max-abs with the same iteration count; the
converged lexicographic solution 1e-6.
"""
from dataclasses import replace

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import oracle as orc  # noqa: E402
import synth  # noqa: E402
from paper_2111_11866_amd import binding as B  # noqa: E402

DEV = "cuda"


def T(a, dtype=None):
    a = np.ascontiguousarray(a)
    t = torch.from_numpy(a).to(DEV)
    return t if dtype is None else t.to(dtype)


def H(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def assert_same(got, ref, what=""):
    """bit-exact comparison with a compact report"""
    got, ref = np.asarray(got), np.asarray(ref)
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    bad = got != ref
    if bad.any():
        d = np.abs(got.astype(np.float64) - ref.astype(np.float64))
        idx = np.unravel_index(np.argmax(d), d.shape)
        raise AssertionError(f"{what}: {int(bad.sum())} of {bad.size} differ; max |diff| {d.max():.3e} "
                             f"at {idx}: got {got[idx]!r} ref {ref[idx]!r}")


def assert_close(got, ref, atol, what=""):
    d = np.abs(np.asarray(got) - np.asarray(ref))
    if not (d <= atol).all():
        idx = np.unravel_index(np.argmax(d), d.shape)
        raise AssertionError(f"{what}: max |diff| {d.max():.3e} > {atol:.1e} at {idx}")


def orc_pp(p: B.PrepareParams):
    return orc.PrepareParams(K=p.K, delta=p.delta, vartheta=p.vartheta, lam=p.lam, ball_r=p.ball_r,
                             smooth_tau=p.smooth_tau, smooth_steps=p.smooth_steps,
                             smooth_omega=p.smooth_omega, smooth_tol=p.smooth_tol)


# ----------------------------------------------------------------- fixtures


@pytest.fixture(scope="module")
def cfg1():
    img = synth.spheres_cfg1()
    pp = B.PrepareParams()
    sp = B.StepParams()
    prep = orc.prepare(img.n, img.image, img.centres, orc_pp(pp))
    u0 = orc.init_u(img.n, img.seeds, 1.0, 0.0)
    w = orc.rescale(img.n, u0, img.centres, sp.ball_r, prep["owner"])
    return dict(img=img, pp=pp, sp=sp, prep=prep, u0=u0, w0=w)


def gpu_prepare(img, pp):
    n = img.n
    image = T(img.image)
    cen, nc = B.centres_tensor(img.centres)
    G = torch.empty((4,) + B.padded_shape(n), dtype=torch.float64, device=DEV)
    owner = torch.empty(B.interior_shape(n), dtype=torch.int32, device=DEV)
    ws = B.alloc_workspace(n, nc)
    rc = B.prepare_g(n, 1.0, image, cen, nc, pp, G, owner, ws)
    return rc, G, owner, ws, cen, nc


# ---------------------------------------------------------------- preparation


def test_library_exports():
    import ctypes

    L = B.lib()
    for name in B.EXPORTED:
        assert hasattr(L, name)
    assert ctypes.sizeof(B.StepParamsC) == 80 and ctypes.sizeof(B.PrepareParamsC) == 80


def test_prepare_cfg1(cfg1):
    rc, G, owner, ws, cen, nc = gpu_prepare(cfg1["img"], cfg1["pp"])
    assert rc == 0
    assert_same(H(owner), cfg1["prep"]["owner"], "owner")
    assert_close(H(G), cfg1["prep"]["G"], 1e-12, "G")


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_prepare_nuclei_window(dtype):
    img = synth.window_job((33, 29, 26, 4), 1000, 100000)
    scale = 1.0 / 255.0
    if dtype == "f32":
        src = img.image.astype(np.float32)
    else:
        src = img.image
    pp = B.PrepareParams(ball_r=8.0, image_scale=scale)
    gimg = synth.Image4D(n=img.n, image=src, centres=img.centres, seeds=img.seeds)
    rc, G, owner, ws, cen, nc = gpu_prepare(gimg, pp)
    I0 = src.astype(np.float64) * scale
    prep = orc.prepare(img.n, I0, img.centres, orc_pp(pp))
    assert rc == 0
    assert_same(H(owner), prep["owner"], "owner")
    assert_close(H(G), prep["G"], 1e-12, "G")


def test_prepare_many_overlapping_balls():
    """dense, overlapping balls: nearest-centre ownership with ties."""
    rng = np.random.default_rng(4)
    n = (20, 18, 16, 3)
    cs = np.zeros(30, dtype=B.CENTRE_DTYPE)
    cs["x"] = np.round(rng.uniform(0, 19, 30) * 2) / 2
    cs["y"] = np.round(rng.uniform(0, 17, 30) * 2) / 2
    cs["z"] = np.round(rng.uniform(0, 15, 30) * 2) / 2
    cs["frame"] = rng.integers(0, 3, 30)
    image = rng.uniform(0, 1, size=B.interior_shape(n))
    img = synth.Image4D(n=n, image=image, centres=cs, seeds=cs)
    pp = B.PrepareParams(ball_r=4.0, K=50.0)
    rc, G, owner, ws, cen, nc = gpu_prepare(img, pp)
    prep = orc.prepare(n, image, cs, orc_pp(pp))
    assert_same(H(owner), prep["owner"], "owner")
    assert_close(H(G), prep["G"], 1e-12, "G")


@pytest.mark.parametrize("R", [0.0, 6.0])
def test_init_u_bitexact(R):
    rng = np.random.default_rng(int(R) + 3)
    n = (21, 17, 13, 4)
    seeds = np.zeros(9, dtype=B.CENTRE_DTYPE)
    seeds["x"] = rng.uniform(0, 20, 9)
    seeds["y"] = rng.uniform(0, 16, 9)
    seeds["z"] = rng.uniform(0, 12, 9)
    seeds["frame"] = [0, 0, 1, 1, 1, 2, 2, 0, 1]
    st, ns = B.centres_tensor(seeds)
    u = torch.full(B.padded_shape(n), 7.0, dtype=torch.float64, device=DEV)
    B.init_u(n, 1.0, st, ns, 1.0, R, u)
    ref = orc.init_u(n, seeds, 1.0, R)
    assert_same(H(u), ref, "u0")


def test_rescale_bitexact(cfg1):
    img = cfg1["img"]
    n = img.n
    cen, nc = B.centres_tensor(img.centres)
    owner = T(cfg1["prep"]["owner"])
    u = T(cfg1["u0"])
    ws = B.alloc_workspace(n, nc)
    B.rescale(n, 1.0, cen, nc, cfg1["sp"].ball_r, owner, u, ws)
    assert_same(H(u), cfg1["w0"], "rescaled u0")


# ------------------------------------------------------------------ assembly


def test_assemble_matches_oracle(cfg1):
    img, sp = cfg1["img"], cfg1["sp"]
    n = img.n
    G = T(cfg1["prep"]["G"])
    w = T(cfg1["w0"])
    coef = torch.empty(B.interior_shape(n) + (8,), dtype=torch.float64, device=DEV)
    b = torch.empty(B.interior_shape(n), dtype=torch.float64, device=DEV)
    B.assemble(n, 1.0, G, w, sp, coef, b)
    c_ref, b_ref = orc.assemble(n, cfg1["prep"]["G"], cfg1["w0"], 1.0, sp.eps, sp.tau)
    c = H(coef)
    assert (np.abs(c - c_ref) <= 1e-13 * np.maximum(1.0, np.abs(c_ref))).all()
    assert np.abs(H(b) - b_ref).max() <= 1e-13


def test_assemble_dirichlet_ghosts_and_h():
    """non-zero Dirichlet ghosts and h != 1 enter b and the gradients."""
    rng = np.random.default_rng(8)
    n = (9, 7, 6, 5)
    h = 0.37
    G = rng.uniform(0.05, 1, size=(4,) + B.padded_shape(n))
    w = rng.uniform(-1, 1, size=B.padded_shape(n))
    sp = B.StepParams(eps=0.05, tau=0.02)
    coef = torch.empty(B.interior_shape(n) + (8,), dtype=torch.float64, device=DEV)
    b = torch.empty(B.interior_shape(n), dtype=torch.float64, device=DEV)
    B.assemble(n, h, T(G), T(w), sp, coef, b)
    c_ref, b_ref = orc.assemble(n, G, w, h, sp.eps, sp.tau)
    assert (np.abs(H(coef) - c_ref) <= 1e-13 * np.maximum(1.0, np.abs(c_ref))).all()
    assert np.abs(H(b) - b_ref).max() <= 1e-13


def test_prepare_wide_rows():
    """A 260-voxel row (two coefficient tiles of 128 slots and a ragged third)
    takes the wide-row forms of the preparation kernels: owner map bit-exact,
    G within 1e-12 of the oracle."""
    n = (260, 40, 12, 3)
    img = synth.window_job(n, 4242, 4343)
    pp = B.PrepareParams(ball_r=8.0, image_scale=1.0 / 255.0)
    rc, G, owner, ws, cen, nc = gpu_prepare(img, pp)
    prep = orc.prepare(n, img.image.astype(np.float64) / 255.0, img.centres, orc_pp(pp))
    assert rc == 0
    assert_same(H(owner), prep["owner"], "owner")
    assert_close(H(G), prep["G"], 1e-12, "G")


# --------------------------------------------------------------------- solve


RAGGED = [(1, 1, 1, 1), (2, 1, 1, 1), (3, 2, 2, 2), (5, 4, 3, 3), (7, 6, 5, 4), (4, 3, 3, 2),
          (130, 3, 2, 2), (129, 4, 2, 3), (64, 5, 3, 2), (33, 9, 7, 3),
          # wide rows with more frames than the sweep holds back before writing
          # (8), not a multiple of it, and more rows than one block (16)
          (133, 37, 5, 13), (257, 19, 3, 9)]


def random_system(n, seed, tau=0.5):
    rng = np.random.default_rng(seed)
    G = rng.uniform(0.05, 1, size=(4,) + B.padded_shape(n))
    w = rng.uniform(0, 1, size=B.padded_shape(n))
    w[0] = w[-1] = 0; w[:, 0] = w[:, -1] = 0; w[:, :, 0] = w[:, :, -1] = 0; w[..., 0] = w[..., -1] = 0
    coef, b = orc.assemble(n, G, w, 1.0, 1e-2, tau)
    return G, w, coef, b


@pytest.mark.parametrize("n", RAGGED)
def test_solve_fixed_iterations(n):
    """Red-black iterates do not depend on the order inside a phase, so the
    GPU's iterate after k sweeps equals the oracle's."""
    G, w, coef, b = random_system(n, sum(n))
    for k in (1, 2, 7):
        sp = B.StepParams(omega=1.3, fixed_iters=k, rescale=False)
        u = T(w)
        ws = B.alloc_workspace(n)
        r = B.solve(n, 1.0, T(coef), T(b), u, sp, ws)
        ref, it, rr, st = orc.sor(n, coef, b, w, 1.3, 0.0, k, orc.RB)
        assert r["iterations"] == k
        assert np.abs(H(u)[1:-1, 1:-1, 1:-1, 1:-1] - ref[1:-1, 1:-1, 1:-1, 1:-1]).max() <= 1e-12
        assert abs(r["rel_res"] - rr) <= 1e-9 * max(rr, 1e-300) + 1e-15


@pytest.mark.parametrize("n", [(3, 3, 2, 2), (4, 3, 3, 2), (5, 4, 2, 3)])
def test_solve_matches_dense_lu(n):
    G, w, coef, b = random_system(n, 3 * sum(n))
    A, bb = orc.dense_system(n, coef, b)
    x = np.linalg.solve(A, bb).reshape(B.interior_shape(n))
    u = T(w)
    r = B.solve(n, 1.0, T(coef), T(b), u, B.StepParams(omega=1.4, tol=1e-15, rescale=False), B.alloc_workspace(n))
    assert r["status"] == 0
    assert np.abs(H(u)[1:-1, 1:-1, 1:-1, 1:-1] - x).max() <= 1e-12


def rerun_if_split(n, coef, b, w, sp, ws, r, u, it, omega, tol):
    """When the GPU and the oracle stop at different iterations, the iterate
    k = min of the two passed the stopping rule on one side only, so its
    residual must lie at the threshold (relative 1e-6); then the GPU reruns at
    the oracle's count and its iterate is returned for comparison."""
    if r["iterations"] == it:
        return u
    kmin = min(r["iterations"], it)
    _, _, rk, _ = orc.sor(n, coef, b, w, omega, 0.0, kmin, orc.RB)
    assert abs(rk / tol - 1) < 1e-6, (r, it, rk)
    u2 = T(w)
    r2 = B.solve(n, 1.0, T(coef), T(b), u2, replace(sp, fixed_iters=it), ws)
    assert r2["iterations"] == it
    return u2


@pytest.mark.parametrize("n", RAGGED)
def test_solve_tolerance_same_iterations(n):
    G, w, coef, b = random_system(n, 5 * sum(n))
    sp = B.StepParams(omega=1.5, tol=1e-9, rescale=False)
    u = T(w)
    ws = B.alloc_workspace(n)
    r = B.solve(n, 1.0, T(coef), T(b), u, sp, ws)
    ref, it, rr, st = orc.sor(n, coef, b, w, 1.5, 1e-9, 10000, orc.RB)
    u = rerun_if_split(n, coef, b, w, sp, ws, r, u, it, 1.5, 1e-9)
    assert np.abs(H(u)[1:-1, 1:-1, 1:-1, 1:-1] - ref[1:-1, 1:-1, 1:-1, 1:-1]).max() <= 1e-12


@pytest.mark.parametrize("n,check", [((5, 4, 3, 3), 3), ((33, 9, 7, 3), 4), ((130, 3, 2, 2), 5)])
def test_solve_check_every(n, check):
    """With check_every = c the stopping rule is tested at k = 0, c, 2c, ...:
    the GPU stops at the oracle's iteration (a multiple of c) with its iterate."""
    G, w, coef, b = random_system(n, 7 * sum(n))
    sp = B.StepParams(omega=1.5, tol=1e-9, rescale=False, check_every=check)
    u = T(w)
    ws = B.alloc_workspace(n)
    r = B.solve(n, 1.0, T(coef), T(b), u, sp, ws)
    ref, it, rr, st = orc.sor(n, coef, b, w, 1.5, 1e-9, 10000, orc.RB, check)
    assert it % check == 0 and r["iterations"] % check == 0
    u = rerun_if_split(n, coef, b, w, sp, ws, r, u, it, 1.5, 1e-9)
    assert np.abs(H(u)[1:-1, 1:-1, 1:-1, 1:-1] - ref[1:-1, 1:-1, 1:-1, 1:-1]).max() <= 1e-12


@pytest.mark.parametrize("tau", [5.0, 200.0])
@pytest.mark.parametrize("precision", [B.FP64, B.MIXED])
def test_stiff_step(tau, precision):
    """A large time step makes the rows barely diagonally dominant (tau = 200:
    the off-diagonal weight of a row is ~0.999 of its diagonal) and SOR slow.
    The FP64 step and the mixed step (BF16 coefficients, refined in FP64) both
    reach their rule and lie within the sum of the two tolerances times
    ||b||_2 of the oracle converged to 1e-13 (||A^-1||_inf <= 1)."""
    n = (12, 10, 8, 4)
    rng = np.random.default_rng(77)
    G = rng.uniform(0.05, 1, size=(4,) + B.padded_shape(n))
    w = np.zeros(B.padded_shape(n))
    w[1:-1, 1:-1, 1:-1, 1:-1] = rng.uniform(0, 1, size=B.interior_shape(n))
    ref = orc.step(n, G, w, None, None, orc.StepParams(tau=tau, omega=1.9, tol=1e-13, rescale=False), orc.RB)
    assert ref["status"] == 0
    tol = 1e-11
    sp = B.StepParams(tau=tau, omega=1.9, tol=tol, max_iter=200000, rescale=False, precision=precision,
                      refine_tol=tol, inner_sweeps=20)
    u = T(w)
    r = B.step(n, 1.0, T(G), None, 0, None, u, sp, B.alloc_workspace(n, 0, precision))
    assert r["status"] == 0 and r["rel_res"] <= tol, r
    err = np.abs(H(u) - ref["u_resc"]).max()
    assert err <= (tol + 1e-13) * r["bnorm"] * (1 + 1e-6), (err, r)


# ---------------------------------------------------------------------- step


def step_gpu(n, G, w, cen, nc, owner, sp, ws):
    u = T(w)
    r = B.step(n, 1.0, G, cen, nc, owner, u, sp, ws)
    return H(u), r


def test_step_teacher_forced_cfg1(cfg1):
    """Config 1, 20 steps: each step starts both sides from the oracle's
    u^{resc;n-1}; the GPU result equals the red-black oracle to 1e-10 with the
    same iteration count (fixed-count rerun when R_k lies within 1e-6 of the
    threshold)."""
    img, sp = cfg1["img"], cfg1["sp"]
    n = img.n
    G_np = cfg1["prep"]["G"]
    G = T(G_np)
    owner = T(cfg1["prep"]["owner"])
    cen, nc = B.centres_tensor(img.centres)
    ws = B.alloc_workspace(n, nc)
    w = cfg1["w0"]
    osp = orc.StepParams()
    worst = 0.0
    for s in range(20):
        rec = orc.step(n, G_np, w, img.centres, cfg1["prep"]["owner"], osp, orc.RB)
        ug, r = step_gpu(n, G, w, cen, nc, owner, sp, ws)
        assert r["status"] == 0
        if r["iterations"] != rec["iterations"]:
            # the iterate min(k_gpu, k_oracle) passed the rule on one side only:
            # its residual must lie at the threshold before a fixed-count rerun
            k = rec["iterations"]
            kmin = min(k, r["iterations"])
            near = orc.step(n, G_np, w, img.centres, cfg1["prep"]["owner"], osp, orc.RB, fixed_iters=kmin)
            assert abs(near["rel_res"] / osp.tol - 1) < 1e-6, (s, r, k, near["rel_res"])
            rec = orc.step(n, G_np, w, img.centres, cfg1["prep"]["owner"], osp, orc.RB, fixed_iters=k)
            ug, r = step_gpu(n, G, w, cen, nc, owner, B.StepParams(fixed_iters=k), ws)
        err = np.abs(ug - rec["u_resc"]).max()
        worst = max(worst, err)
        assert err <= 1e-10, (s, err)
        w = rec["u_resc"]
    print("worst per-step max-abs vs oracle:", worst)


def test_step_teacher_forced_wide_window():
    """A nuclei window with wide rows (the two-cell sweep in 16-row blocks),
    27 rows, 11 frames (a held-back write group of 8 frames and a tail of 3),
    balls and rescale: the oracle's preparation, then 4 steps each from the
    oracle's u^{resc;n-1}, the GPU within 1e-10 of the red-black oracle."""
    img = synth.window_job((131, 27, 13, 11), 7, 70007)
    pp = B.PrepareParams(ball_r=8.0, image_scale=1.0 / 255.0)
    n = img.n
    prep = orc.prepare(n, img.image.astype(np.float64) / 255.0, img.centres, orc_pp(pp))
    sp = B.StepParams(omega=1.6)
    osp = orc.StepParams(omega=1.6)
    G_np = prep["G"]
    G = T(G_np)
    owner = T(prep["owner"])
    cen, nc = B.centres_tensor(img.centres)
    ws = B.alloc_workspace(n, nc)
    w = orc.rescale(n, orc.init_u(n, img.seeds, 1.0, 0.0), img.centres, sp.ball_r, prep["owner"])
    for s in range(4):
        rec = orc.step(n, G_np, w, img.centres, prep["owner"], osp, orc.RB)
        ug, r = step_gpu(n, G, w, cen, nc, owner, sp, ws)
        assert r["status"] == 0
        if r["iterations"] != rec["iterations"]:
            k = rec["iterations"]
            kmin = min(k, r["iterations"])
            near = orc.step(n, G_np, w, img.centres, prep["owner"], osp, orc.RB, fixed_iters=kmin)
            assert abs(near["rel_res"] / osp.tol - 1) < 1e-6, (s, r, k, near["rel_res"])
            rec = orc.step(n, G_np, w, img.centres, prep["owner"], osp, orc.RB, fixed_iters=k)
            ug, r = step_gpu(n, G, w, cen, nc, owner, replace(sp, fixed_iters=k), ws)
        assert r["iterations"] >= 2
        err = np.abs(ug - rec["u_resc"]).max()
        assert err <= 1e-10, (s, err)
        w = rec["u_resc"]


def test_step_vs_converged_lexicographic(cfg1):
    img, sp = cfg1["img"], cfg1["sp"]
    n = img.n
    G_np = cfg1["prep"]["G"]
    cen, nc = B.centres_tensor(img.centres)
    ws = B.alloc_workspace(n, nc)
    ug, r = step_gpu(n, T(G_np), cfg1["w0"], cen, nc, T(cfg1["prep"]["owner"]), sp, ws)
    lex = orc.step(n, G_np, cfg1["w0"], img.centres, cfg1["prep"]["owner"],
                   orc.StepParams(tol=1e-13), orc.LEX)
    assert np.abs(ug - lex["u_resc"]).max() <= 1e-6


def test_free_running_trajectory_cfg1(cfg1):
    """20 steps on each side without teacher forcing (reported; bounded)."""
    img, sp = cfg1["img"], cfg1["sp"]
    job = B.Job(img.n, img.image, img.centres, img.seeds)
    assert job.prepare(cfg1["pp"]) == 0
    job.init(v=1.0, R=0.0, ball_r=sp.ball_r)
    out = orc.run(img.n, img.image, img.centres, img.seeds, orc_pp(cfg1["pp"]), orc.StepParams(), steps=20)
    errs = []
    for s in range(20):
        job.step(sp)
        errs.append(float(np.abs(H(job.u) - out["steps"][s]["u_resc"]).max()))
    print("free-running max-abs per step:", errs)
    assert max(errs) <= 1e-6


def test_step_constant_is_fixed_point():
    n = (10, 9, 8, 4)
    G = torch.rand((4,) + B.padded_shape(n), dtype=torch.float64, device=DEV) * 0.9 + 0.1
    u = torch.full(B.padded_shape(n), 0.3125, dtype=torch.float64, device=DEV)
    ws = B.alloc_workspace(n)
    r = B.step(n, 1.0, G, None, 0, None, u, B.StepParams(rescale=False), ws)
    assert r["iterations"] == 0 and r["status"] == 0
    assert (H(u) == 0.3125).all()


def test_step_tau_zero_is_identity():
    rng = np.random.default_rng(1)
    n = (8, 7, 6, 3)
    w = rng.uniform(0, 1, size=B.padded_shape(n))
    u = T(w)
    r = B.step(n, 1.0, torch.ones((4,) + B.padded_shape(n), dtype=torch.float64, device=DEV), None, 0, None,
               u, B.StepParams(tau=0.0, rescale=False), B.alloc_workspace(n))
    assert r["iterations"] == 0
    assert np.array_equal(H(u), w)


def test_step_axis_permutation_equivariance():
    """With uniform h the scheme treats the four axes alike (Sec. 3.2.2): for
    each of the 24 axis permutations, permuting u and G (G's face components
    with their axes) permutes the step's result.  The red-black colour
    (i+j+k+l) is invariant, so fixed-count iterates agree up to the order of
    the floating-point sums: 1e-13."""
    import itertools

    n = (7, 6, 5, 4)
    rng = np.random.default_rng(21)
    G = rng.uniform(0.05, 1.0, size=(4,) + B.padded_shape(n))
    w = np.zeros(B.padded_shape(n))
    w[1:-1, 1:-1, 1:-1, 1:-1] = rng.uniform(0.0, 1.0, size=B.interior_shape(n))
    sp = B.StepParams(fixed_iters=6, rescale=False)
    base, _ = step_gpu(n, T(G), w, None, 0, None, sp, B.alloc_workspace(n))
    worst = 0.0
    for perm in itertools.permutations(range(4)):
        # new axis d takes old axis perm[d]; numpy axis a holds axis 3 - a
        axes = [3 - perm[3 - a] for a in range(4)]
        n2 = tuple(n[perm[d]] for d in range(4))
        w2 = np.ascontiguousarray(w.transpose(axes))
        G2 = np.ascontiguousarray(np.stack([G[perm[d]].transpose(axes) for d in range(4)]))
        u2, r = step_gpu(n2, T(G2), w2, None, 0, None, sp, B.alloc_workspace(n2))
        assert r["iterations"] == 6
        back = u2.transpose(np.argsort(axes))
        worst = max(worst, float(np.abs(back - base).max()))
    assert worst <= 1e-13, worst


# --------------------------------------------------------------- error paths


def test_not_converged_status():
    G, w, coef, b = random_system((6, 5, 4, 3), 2)
    u = T(w)
    r = B.solve((6, 5, 4, 3), 1.0, T(coef), T(b), u, B.StepParams(tol=1e-14, max_iter=1, rescale=False),
                B.alloc_workspace((6, 5, 4, 3)))
    assert r["status"] == B.NOT_CONVERGED and r["iterations"] == 1
    ref, *_ = orc.sor((6, 5, 4, 3), coef, b, w, 1.5, 0.0, 1, orc.RB)
    assert np.abs(H(u) - ref)[1:-1, 1:-1, 1:-1, 1:-1].max() <= 1e-12


def test_nonfinite_input_reported():
    n = (6, 5, 4, 3)
    G, w, coef, b = random_system(n, 3)
    b = b.copy()
    b[1, 1, 1, 1] = np.nan
    with pytest.raises(B.Subsurf4dError) as e:
        B.solve(n, 1.0, T(coef), T(b), T(w), B.StepParams(rescale=False), B.alloc_workspace(n))
    assert e.value.status == B.ENONFINITE


def test_bad_arguments_rejected():
    n = (6, 5, 4, 3)
    G, w, coef, b = random_system(n, 3)
    small = torch.empty(1024, dtype=torch.uint8, device=DEV)
    with pytest.raises(B.Subsurf4dError) as e:
        B.solve(n, 1.0, T(coef), T(b), T(w), B.StepParams(rescale=False), small)
    assert e.value.status == B.EWORKSPACE
    with pytest.raises(B.Subsurf4dError) as e:
        B.solve((0, 5, 4, 3), 1.0, T(coef), T(b), T(w), B.StepParams(rescale=False), small)
    assert e.value.status == B.ESHAPE
    with pytest.raises(B.Subsurf4dError) as e:
        B.solve(n, 1.0, T(coef), T(b), T(w), B.StepParams(omega=2.0, rescale=False), B.alloc_workspace(n))
    assert e.value.status == B.EINVAL
    # iteration caps far from INT_MAX (pass counters run to max_iter + 1)
    for bad in (dict(max_iter=(1 << 30) + 1), dict(max_iter=2 ** 31 - 1), dict(fixed_iters=(1 << 30) + 1),
                dict(precision=B.MIXED, inner_sweeps=1025)):
        with pytest.raises(B.Subsurf4dError) as e:
            B.solve(n, 1.0, T(coef), T(b), T(w), B.StepParams(rescale=False, **bad), B.alloc_workspace(n))
        assert e.value.status == B.EINVAL, bad
    im = synth.window_job(n, 5, 6)
    job = B.Job(n, im.image, im.centres, im.seeds, precision=B.FP64)
    with pytest.raises(B.Subsurf4dError) as e:
        job.prepare(B.PrepareParams(image_scale=1.0 / 255.0, smooth_max_iter=2 ** 31 - 1))
    assert e.value.status == B.EINVAL


def test_deterministic_repeat(cfg1):
    img, sp = cfg1["img"], cfg1["sp"]
    n = img.n
    cen, nc = B.centres_tensor(img.centres)
    ws = B.alloc_workspace(n, nc)
    a, ra = step_gpu(n, T(cfg1["prep"]["G"]), cfg1["w0"], cen, nc, T(cfg1["prep"]["owner"]), sp, ws)
    b, rb = step_gpu(n, T(cfg1["prep"]["G"]), cfg1["w0"], cen, nc, T(cfg1["prep"]["owner"]), sp, ws)
    assert np.array_equal(a, b) and ra == rb


def test_stream_probe_sums_chunks():
    """The read-dominated bandwidth probe computes dst = sum of its source
    chunks (writes=1), or per-block partial sums whose total is the sum of the
    whole source (writes=0); integer-valued data, so both are exact."""
    n = 1 << 16
    src = torch.arange(3 * 2 * n, dtype=torch.float64, device=DEV)
    dst = torch.empty(2 * n, dtype=torch.float64, device=DEV)
    ms = B.stream_probe(src, dst, 3, reps=2)
    assert ms > 0.0
    want = src.view(3, 2 * n).sum(0)
    assert torch.equal(dst, want)
    g = B.stream_probe_blocks(dst)
    assert g == n // 1024
    dst.fill_(-1.0)
    ms = B.stream_probe(src, dst, 3, writes=0, reps=2)
    assert ms > 0.0
    assert float(dst[: 2 * g].sum()) == float(src.sum())
    assert bool((dst[2 * g:] == -1.0).all())


def test_red_phase_reads_only_black():
    """Red-black ordering (Sec. 3.2.2): the red half-sweep reads only black
    neighbours.  With omega = 1 one iteration's result does not depend on the
    red values of the initial guess: poisoning them (1e100) leaves the iterate,
    its iteration count and its residual bitwise unchanged, while poisoning
    the black values changes the result."""
    n = (33, 9, 7, 3)
    G, w, coef, b = random_system(n, 99)
    idx = np.indices(B.padded_shape(n)).sum(0)          # l + k + j + i
    interior = np.zeros(B.padded_shape(n), dtype=bool)
    interior[1:-1, 1:-1, 1:-1, 1:-1] = True
    red = interior & (idx % 2 == 0)
    sp = B.StepParams(omega=1.0, fixed_iters=1, rescale=False)
    ws = B.alloc_workspace(n)
    u0 = w.copy(); u0[red] = 0.0
    a = T(u0)
    ra = B.solve(n, 1.0, T(coef), T(b), a, sp, ws)
    up = w.copy(); up[red] = 1e100
    p = T(up)
    rp = B.solve(n, 1.0, T(coef), T(b), p, sp, ws)
    assert np.array_equal(H(a)[interior], H(p)[interior]) and ra["iterations"] == rp["iterations"] == 1
    assert ra["rel_res"] == rp["rel_res"]
    ub = u0.copy(); ub[interior & ~red] = 1e100
    q = T(ub)
    B.solve(n, 1.0, T(coef), T(b), q, sp, ws)
    assert not np.array_equal(H(q)[interior], H(a)[interior])


def test_checkpoint_resume_bit_identical(cfg1, tmp_path):
    """20 steps in one go equal 10 steps, a checkpoint to disk, a fresh job
    resumed from it, and 10 more steps, bitwise."""
    img, sp = cfg1["img"], cfg1["sp"]
    full = B.Job(img.n, img.image, img.centres, img.seeds)
    assert full.prepare(cfg1["pp"]) == 0
    full.init(v=1.0, R=0.0, ball_r=sp.ball_r)
    for _ in range(20):
        full.step(sp)
    half = B.Job(img.n, img.image, img.centres, img.seeds)
    half.prepare(cfg1["pp"])
    half.init(v=1.0, R=0.0, ball_r=sp.ball_r)
    for _ in range(10):
        half.step(sp)
    path = str(tmp_path / "job.npz")
    half.save(path)
    del half
    resumed = B.Job(img.n, img.image, img.centres, img.seeds)
    resumed.load(path)
    for _ in range(10):
        resumed.step(sp)
    assert torch.equal(resumed.u, full.u)


def test_sweep_forms_and_grids_give_the_same_bits(monkeypatch):
    """Every red-black sweep form (row tiles, one-cell and two-cell frame
    marching, 8-row blocks), every grid size of the frame-marching sweeps and
    both assembly loadings and store kinds leave the same iterate, bit for
    bit: red-black SOR does not depend on the order of updates within a
    colour, the fixed-count solve tests no stopping rule, and each cell's
    arithmetic is the same in every form.  Also the mixed step at several
    grids of its FP32 sweep: same iterate, passes and inner iterations."""
    forms = [{}, {"SUBSURF4D_SWEEP": "r"}, {"SUBSURF4D_SWEEP": "t"}, {"SUBSURF4D_SWEEP": "8"},
             {"SUBSURF4D_SWEEP": "p"}, {"SUBSURF4D_SWEEP": "d"}, {"SUBSURF4D_SWEEP": "D"},
             {"SUBSURF4D_SWEEP_GRID": "13"}, {"SUBSURF4D_SWEEP_GRID": "100"}, {"SUBSURF4D_SWEEP_GRID": "300"},
             {"SUBSURF4D_ASM_PREFETCH": "0"}, {"SUBSURF4D_ASM_NT": "0"}]
    keys = {k for f in forms for k in f}
    # two-cell rows (>= 64 slots), ragged in every axis; the second with 13
    # frames (a held-back group of 8 and a tail of 5) and 37 rows (3 blocks)
    for n in ((131, 10, 6, 4), (133, 37, 5, 13)):
        rng = np.random.default_rng(77)
        G = T(rng.uniform(0.05, 1.0, size=(4,) + B.padded_shape(n)))
        w = np.zeros(B.padded_shape(n))
        w[1:-1, 1:-1, 1:-1, 1:-1] = rng.uniform(0.0, 1.0, size=B.interior_shape(n))
        ws = B.alloc_workspace(n, 0, B.MIXED)
        sp = B.StepParams(fixed_iters=9, rescale=False, omega=1.7)
        ref = None
        for f in forms:
            for k in keys:
                monkeypatch.delenv(k, raising=False)
            for k, v in f.items():
                monkeypatch.setenv(k, v)
            u, r = step_gpu(n, G, w, None, 0, None, sp, ws)
            assert r["iterations"] == 9, (n, f, r)
            if ref is None:
                ref = u
            else:
                assert np.array_equal(u, ref), (n, f)
        for k in keys:
            monkeypatch.delenv(k, raising=False)
    n = (131, 10, 6, 4)
    rng = np.random.default_rng(77)
    G = T(rng.uniform(0.05, 1.0, size=(4,) + B.padded_shape(n)))
    w = np.zeros(B.padded_shape(n))
    w[1:-1, 1:-1, 1:-1, 1:-1] = rng.uniform(0.0, 1.0, size=B.interior_shape(n))
    ws = B.alloc_workspace(n, 0, B.MIXED)
    msp = B.StepParams(precision=B.MIXED, rescale=False, refine_tol=1e-11, inner_sweeps=6, omega=1.7)
    mref = None
    for g in (None, "20", "75", "250"):
        if g is None:
            monkeypatch.delenv("SUBSURF4D_SWEEP_GRID", raising=False)
        else:
            monkeypatch.setenv("SUBSURF4D_SWEEP_GRID", g)
        u, r = step_gpu(n, G, w, None, 0, None, msp, ws)
        assert r["status"] == 0
        if mref is None:
            mref = (u, r["outer"], r["iterations"])
        else:
            assert np.array_equal(u, mref[0]) and r["outer"] == mref[1] and r["iterations"] == mref[2], g
    monkeypatch.delenv("SUBSURF4D_SWEEP_GRID", raising=False)
