"""The allocation-free step (library-held device scratch) against the step
with a caller workspace: the same kernels on the same inputs, so the results
are bitwise equal; two calls in a row, the second on a smaller grid, then a
grid beyond the scratch is refused."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import synth  # noqa: E402
from paper_2111_11866_amd import binding as B  # noqa: E402


def _job(n, seed):
    img = synth.spheres_cfg1(n=n, n_spheres=1, geom_seed=seed, noise_seed=seed + 1)
    job = B.Job(n, img.image, img.centres, img.seeds, precision=B.MIXED)
    assert job.prepare(B.PrepareParams()) == 0
    job.init(v=1.0, R=0.0, ball_r=8.0)
    return job


@pytest.mark.parametrize("precision", [B.FP64, B.MIXED])
def test_step_noalloc_matches_step(precision):
    sp = B.StepParams(precision=precision, refine_tol=1e-10, inner_sweeps=8)
    for n, seed in (((24, 24, 24, 8), 1), ((20, 18, 16, 4), 5)):     # second call: smaller grid
        assert B.workspace_bytes(n, 8, precision) <= B.NOALLOC_SCRATCH_BYTES
        job = _job(n, seed)
        u0 = job.u.clone()
        ref = B.step(n, 1.0, job.G, job.centres, job.nc, job.owner, job.u, sp, job.ws)
        want = job.u.clone()
        job.u.copy_(u0)
        got = B.step_noalloc(n, 1.0, job.G, job.centres, job.nc, job.owner, job.u, sp)
        torch.cuda.synchronize()
        assert got == ref, (n, got, ref)
        assert torch.equal(job.u, want), (n, float((job.u - want).abs().max()))


def test_step_noalloc_refuses_large_grids():
    n = (96, 96, 96, 12)
    assert B.workspace_bytes(n) > B.NOALLOC_SCRATCH_BYTES
    G = torch.ones((4,) + B.padded_shape(n), dtype=torch.float64, device="cuda")
    u = torch.zeros(B.padded_shape(n), dtype=torch.float64, device="cuda")
    with pytest.raises(B.Subsurf4dError) as e:
        B.step_noalloc(n, 1.0, G, None, 0, None, u, B.StepParams(rescale=False))
    assert e.value.status == B.EWORKSPACE
