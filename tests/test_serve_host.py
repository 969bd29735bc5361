"""Host logic of the continuous-batching server, without a GPU: the library
calls are replaced by stand-ins that count steps, so admission order, the HBM
budget, the table size and the latency bookkeeping can be checked on the
CPU."""
import numpy as np
import pytest

from paper_2111_11866_amd import serve as S


class FakeU:
    def __init__(self, n):
        self.a = np.zeros(tuple(v + 2 for v in reversed(n)))

    def cpu(self):
        return self

    def numpy(self):
        return self.a


class FakeJob:
    def __init__(self, n, image, centres, seeds, **kw):
        self.n = tuple(n)
        self.u = FakeU(n)
        self.steps = 0


class FakeImg:
    def __init__(self, n):
        self.n = n
        self.image = None
        self.centres = np.zeros(n[3], dtype=[("x", "f4"), ("y", "f4"), ("z", "f4"), ("frame", "i4")])
        self.seeds = self.centres


@pytest.fixture
def fake_lib(monkeypatch):
    calls = {"prepare": [], "step": []}

    class FakeShared:
        def __init__(self, max_jobs, device="cuda"):
            self.table = None
            self.max_jobs = max_jobs

    def prepare_batched(jobs, pp, v, R, ball_r, table):
        calls["prepare"].append(len(jobs))
        return 0, [0] * len(jobs)

    def step_batched(jobs, sp, table):
        calls["step"].append(len(jobs))
        for j in jobs:
            j.steps += 1
            j.u.a += 1.0
        return 0, [dict(status=0, rel_res=1e-9, outer=2) for _ in jobs]

    monkeypatch.setattr(S, "_Shared", FakeShared)
    monkeypatch.setattr(S.B, "Job", FakeJob)
    monkeypatch.setattr(S.B, "prepare_batched", prepare_batched)
    monkeypatch.setattr(S.B, "step_batched", step_batched)
    monkeypatch.setattr(S, "window_bytes", lambda n, nc: int(np.prod(n)))

    import torch

    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    return calls


def windows(sizes, gap=0.0):
    return [S.Window(jid=q, arrival=q * gap, img=FakeImg(n)) for q, n in enumerate(sizes)]


def server(budget=10 ** 12, max_jobs=4096, steps=3):
    pp, plain, mixed = S.default_params()
    return S.BatchServer(pp, mixed, steps=steps, hbm_budget=budget, max_jobs=max_jobs)


def test_every_job_runs_its_steps_and_returns_a_result(fake_lib):
    ws = windows([(20, 20, 20, 3)] * 5)
    stats = server(steps=4).run(ws, realtime=False)
    assert stats["jobs"] == 5
    for w in ws:
        assert w.result is not None and (w.result == 4.0).all()     # 4 steps, each adds 1
        assert w.finished >= w.admitted >= w.arrival
    assert stats["p99_latency_s"] >= stats["p50_latency_s"] >= 0.0


def test_budget_limits_the_resident_jobs(fake_lib):
    n = (20, 20, 20, 3)
    one = int(np.prod(n))
    ws = windows([n] * 6)
    stats = server(budget=2 * one, steps=2).run(ws, realtime=False)
    assert stats["jobs"] == 6 and stats["max_concurrent"] == 2
    assert max(fake_lib["step"]) <= 2


def test_a_job_larger_than_the_budget_runs_alone(fake_lib):
    big, small = (30, 30, 30, 4), (10, 10, 10, 2)
    ws = windows([big, small])
    stats = server(budget=int(np.prod(small)), steps=2).run(ws, realtime=False)
    assert stats["jobs"] == 2 and stats["max_concurrent"] == 1


def test_table_size_limits_the_batch(fake_lib):
    ws = windows([(12, 12, 12, 2)] * 7)
    stats = server(max_jobs=3, steps=2).run(ws, realtime=False)
    assert stats["jobs"] == 7 and max(fake_lib["step"]) <= 3 and max(fake_lib["prepare"]) <= 3


def test_admission_is_first_come_first_served(fake_lib):
    n = (16, 16, 16, 2)
    ws = windows([n] * 6, gap=0.001)
    server(budget=2 * int(np.prod(n)), steps=2).run(ws, realtime=False)
    adm = [w.admitted for w in sorted(ws, key=lambda w: w.arrival)]
    assert adm == sorted(adm)
