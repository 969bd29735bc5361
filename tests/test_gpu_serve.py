"""Continuous-batching server: results are the same alone and in the mix,
and agree with the plain per-job FP64 path within 1e-6 relative."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from paper_2111_11866_amd import serve as S  # noqa: E402


def test_serving_mix_alone_and_plain():
    pp, plain, mixed = S.default_params()
    wins = S.make_windows(2000.0, 24)
    stats = S.BatchServer(pp, mixed, steps=4, hbm_budget=8 << 30).run(wins)
    assert stats["jobs"] == 24 and stats["max_concurrent"] >= 2
    for q in (0, 7, 23):
        alone = S.make_windows(2000.0, 24)[q]
        alone.arrival = 0.0
        S.BatchServer(pp, mixed, steps=4, hbm_budget=8 << 30).run([alone])
        assert np.array_equal(alone.result, wins[q].result), q
        ref = S.make_windows(2000.0, 24)[q]
        ref.arrival = 0.0
        S.PlainServer(pp, plain, steps=4).run([ref])
        scale = np.abs(ref.result).max()
        assert np.abs(ref.result - wins[q].result).max() <= 1e-6 * scale


def test_serving_budget_makes_jobs_wait_none_dropped():
    pp, plain, mixed = S.default_params()
    wins = S.make_windows(5000.0, 16)
    # a budget below any single window: a job is still admitted when nothing
    # else runs, so the jobs run one after another and none is dropped
    stats = S.BatchServer(pp, mixed, steps=2, hbm_budget=1).run(wins)
    assert stats["jobs"] == 16 and stats["max_concurrent"] == 1
    two = sorted(S.window_bytes(w.img.n, len(w.img.centres)) for w in wins)[:2]
    stats = S.BatchServer(pp, mixed, steps=2, hbm_budget=sum(two) + 1).run(S.make_windows(5000.0, 16))
    assert stats["jobs"] == 16 and stats["max_concurrent"] <= 2


def test_window_forms_within_1e6_of_converged():
    """20-step window jobs: the batched mixed form and the plain FP64 form at
    their default settings both stay within 1e-6 relative of the converged
    solution (FP64 SOR to relative residual 1e-12)."""
    pp, plain, mixed = S.default_params()
    res = {}
    for name, srv in (("batched", S.BatchServer(pp, mixed, steps=20, hbm_budget=8 << 30)),
                      ("plain", S.PlainServer(pp, plain, steps=20)),
                      ("converged", S.PlainServer(pp, S.converged_params(plain), steps=20))):
        wins = S.make_windows(1000.0, 12)
        srv.run(wins, realtime=False)
        res[name] = [w.result for w in wins]
    for form in ("batched", "plain"):
        for q, (a, r) in enumerate(zip(res[form], res["converged"])):
            e = np.abs(a - r).max() / np.abs(r).max()
            assert e <= 1e-6, (form, q, e)


def test_served_windows_match_oracle():
    """Three windows served in a mix of eight (continuous batching, mixed
    precision refined in FP64) against the CPU oracle's run of the same job
    (preparation, initial function, rescale, 4 steps solved to relative
    residual 1e-12): max-abs within 1e-6 of max |u|."""
    import oracle as orc

    pp, plain, mixed = S.default_params()
    wins = S.make_windows(2000.0, 8)
    stats = S.BatchServer(pp, mixed, steps=4, hbm_budget=8 << 30).run(wins)
    assert stats["jobs"] == 8 and stats["max_concurrent"] >= 2
    opp = orc.PrepareParams(K=pp.K, delta=pp.delta, vartheta=pp.vartheta, lam=pp.lam, ball_r=pp.ball_r,
                            smooth_tau=pp.smooth_tau, smooth_steps=pp.smooth_steps,
                            smooth_omega=pp.smooth_omega, smooth_tol=pp.smooth_tol)
    osp = orc.StepParams(eps=mixed.eps, tau=mixed.tau, omega=1.5, tol=1e-12, ball_r=mixed.ball_r)
    for q in (0, 3, 7):
        img = wins[q].img
        I0 = img.image.astype(np.float64) * pp.image_scale
        ref = orc.run(img.n, I0, img.centres, img.seeds, opp, osp, steps=4, v=1.0, R=0.0, record=False)
        u = ref["u_final"]
        err = np.abs(wins[q].result - u).max() / np.abs(u).max()
        assert err <= 1e-6, (q, img.n, err)
