"""Mixed precision (FP32 sweeps on BF16 coefficients, FP64 refinement) against
the FP64 oracle.

Gate: after refinement to ||r||_2 <= 1e-10 ||b||_2 (FP64 residual of the FP64
operator), each step's result differs from the converged FP64 oracle solution
by at most 1e-6 relative to max|u| (max-abs and L2 reported per step).  The
bound follows from ||A^-1||_inf <= 1 (stability section): ||u - u*||_inf <=
||r||_inf <= ||r||_2.
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


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def H(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def cfg1():
    img = synth.spheres_cfg1()
    prep = orc.prepare(img.n, img.image, img.centres, orc.PrepareParams())
    w = orc.rescale(img.n, orc.init_u(img.n, img.seeds, 1.0, 0.0), img.centres, 8.0, prep["owner"])
    return img, prep, w


def test_mixed_steps_cfg1(cfg1):
    """Config-1 grid, 20 steps, each from the oracle's u^{resc;n-1}."""
    img, prep, w = cfg1
    n = img.n
    cen, nc = B.centres_tensor(img.centres)
    owner = T(prep["owner"])
    G = T(prep["G"])
    ws = B.alloc_workspace(n, nc, B.MIXED)
    sp = B.StepParams(precision=B.MIXED, refine_tol=1e-10, inner_sweeps=8)
    worst = 0.0
    report = []
    for s in range(20):
        ref = orc.step(n, prep["G"], w, img.centres, prep["owner"], orc.StepParams(tol=1e-14), orc.RB)
        u = T(w)
        r = B.step(n, 1.0, G, cen, nc, owner, u, sp, ws)
        assert r["status"] == 0 and r["rel_res"] <= 1e-10
        got = H(u)
        scale = np.abs(ref["u_resc"]).max()
        e_max = np.abs(got - ref["u_resc"]).max() / scale
        e_l2 = np.linalg.norm(got - ref["u_resc"]) / np.linalg.norm(ref["u_resc"])
        report.append((s, r["outer"], r["iterations"], float(e_max), float(e_l2)))
        worst = max(worst, e_max)
        assert e_max <= 1e-6, (s, e_max)
        w = ref["u_resc"]
    print("step, refinement passes, inner sweeps, max-abs rel err, L2 rel err:")
    for row in report:
        print(row)


@pytest.mark.parametrize("n", [(5, 4, 3, 3), (7, 6, 5, 4), (33, 9, 7, 3), (130, 5, 3, 3), (129, 6, 4, 3), (257, 4, 3, 2),
                               # degenerate extents (a row with one cell, or none, of a colour) and
                               # a wide grid with 13 frames and rows beyond one tile of rows
                               (1, 1, 1, 1), (2, 1, 1, 1), (1, 3, 1, 2), (3, 2, 2, 1), (130, 1, 1, 1),
                               (133, 20, 3, 13)])
def test_mixed_solve_ragged(n):
    rng = np.random.default_rng(sum(n))
    G = rng.uniform(0.05, 1, size=(4,) + B.padded_shape(n))
    w = rng.uniform(0, 1, size=B.padded_shape(n))
    w[0] = w[-1] = 0; w[:, 0] = w[:, -1] = 0; w[:, :, 0] = w[:, :, -1] = 0; w[..., 0] = w[..., -1] = 0
    ref = orc.step(n, G, w, None, None, orc.StepParams(tol=1e-14, rescale=False), orc.RB)
    u = T(w)
    ws = B.alloc_workspace(n, 0, B.MIXED)
    r = B.step(n, 1.0, T(G), None, 0, None, u, B.StepParams(precision=B.MIXED, rescale=False,
                                                           refine_tol=1e-11, inner_sweeps=6), ws)
    assert r["status"] == 0
    assert np.abs(H(u) - ref["u"]).max() <= 1e-8


def test_mixed_not_converged():
    n = (9, 8, 7, 3)
    rng = np.random.default_rng(3)
    G = T(rng.uniform(0.05, 1, size=(4,) + B.padded_shape(n)))
    w = rng.uniform(0, 1, size=B.padded_shape(n))
    w[0] = w[-1] = 0
    u = T(w)
    r = B.step(n, 1.0, G, None, 0, None, u, B.StepParams(precision=B.MIXED, rescale=False, refine_tol=1e-15,
                                                        inner_sweeps=2, max_iter=4), B.alloc_workspace(n, 0, B.MIXED))
    assert r["status"] == B.NOT_CONVERGED and r["outer"] == 2


def test_mixed_passes_track_fp64_iterations(cfg1):
    """Refinement with m inner red-black sweeps from a zero correction is, in
    exact arithmetic, m steps of the same stationary SOR iteration, so a mixed
    step needs about as many inner sweeps as FP64 SOR needs iterations for the
    same tolerance and relaxation: passes * m <= K_fp64 + 2m on every step of
    the config-1 trajectory (the BF16 coefficients do not slow the refinement
    down as the system sharpens)."""
    img, prep, w = cfg1
    n = img.n
    cen, nc = B.centres_tensor(img.centres)
    owner, G = T(prep["owner"]), T(prep["G"])
    ws = B.alloc_workspace(n, nc, B.MIXED)
    m = 8
    rows = []
    for s in range(20):
        u = T(w)
        r64 = B.step(n, 1.0, G, cen, nc, owner, u, B.StepParams(tol=1e-10, rescale=False), ws)
        u = T(w)
        rmx = B.step(n, 1.0, G, cen, nc, owner, u, B.StepParams(precision=B.MIXED, refine_tol=1e-10,
                                                                 inner_sweeps=m, rescale=False), ws)
        assert r64["status"] == 0 and rmx["status"] == 0
        rows.append((s, r64["iterations"], rmx["outer"]))
        assert rmx["outer"] * m <= r64["iterations"] + 2 * m, rows
        w = orc.step(n, prep["G"], w, img.centres, prep["owner"], orc.StepParams(), orc.RB)["u_resc"]
    print("step, FP64 iterations to 1e-10, mixed passes:", rows)


def test_short_last_pass_cfg1(cfg1):
    """SUBSURF4D_FLAG_SHORT_LAST_PASS only changes how many FP32 iterations
    the later passes run: every step still ends with the FP64 residual at or
    below refine_tol and within the same 1e-6 gate of the converged oracle,
    uses at most one pass's worth of inner iterations more than the
    fixed-length passes on any step, and over the 20 config-1 steps fewer in
    total."""
    img, prep, w = cfg1
    n = img.n
    cen, nc = B.centres_tensor(img.centres)
    owner, G = T(prep["owner"]), T(prep["G"])
    ws = B.alloc_workspace(n, nc, B.MIXED)
    base = B.StepParams(precision=B.MIXED, refine_tol=1e-10, inner_sweeps=8)
    short = B.StepParams(precision=B.MIXED, refine_tol=1e-10, inner_sweeps=8, flags=B.FLAG_SHORT_LAST_PASS)
    tot_base = tot_short = 0
    rows = []
    for s in range(20):
        ref = orc.step(n, prep["G"], w, img.centres, prep["owner"], orc.StepParams(tol=1e-14), orc.RB)
        scale = np.abs(ref["u_resc"]).max()
        u = T(w)
        rb = B.step(n, 1.0, G, cen, nc, owner, u, base, ws)
        u = T(w)
        rs = B.step(n, 1.0, G, cen, nc, owner, u, short, ws)
        assert rb["status"] == 0 and rs["status"] == 0
        assert rs["rel_res"] <= 1e-10
        e_max = np.abs(H(u) - ref["u_resc"]).max() / scale
        assert e_max <= 1e-6, (s, e_max)
        assert rs["iterations"] <= rb["iterations"] + 8, (s, rs, rb)
        tot_base += rb["iterations"]
        tot_short += rs["iterations"]
        rows.append((s, rb["outer"], rb["iterations"], rs["outer"], rs["iterations"], float(e_max)))
        w = ref["u_resc"]
    print("step, passes/iterations fixed, passes/iterations shortened, max-abs rel err:", rows)
    assert tot_short < tot_base, (tot_short, tot_base)
