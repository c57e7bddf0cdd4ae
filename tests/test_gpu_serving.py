"""The serving loop on the GPU: every job's result in the mix equals the job
alone within rounding."""
import sys

import numpy as np
import pytest

from paper_1810_11359_amd import ism, workloads
from paper_1810_11359_amd.serving import GpuExecutor, Job, Scheduler, replay

pytestmark = pytest.mark.gpu


def test_mixed_stream_equals_jobs_alone():
    import torch

    assert torch.cuda.is_available()

    def feasible(room, t60):
        try:
            ism.beta_from_t60(room, t60)
            return True
        except ism.IsmError:
            return False

    reqs = workloads.serving_stream(rate=2000.0, n_jobs=40, seed=11, feasible=feasible)
    # keep the test short: cap each job's RIR length
    jobs = []
    for i, r in enumerate(reqs):
        w = r.workload
        w.t_max = min(w.t_max, 0.25)
        w.t60 = min(w.t60, 0.6) if feasible(w.room, min(w.t60, 0.6)) else w.t60
        jobs.append(Job(i, ism.room_for(w), w.src, w.rcv, r.arrival))
    print(f"[case] serving {len(jobs)} jobs", flush=True)
    ex = GpuExecutor(n_slots=3)
    sch = Scheduler(ex, budget_bytes=2 << 30, n_slots=3, max_batch_jobs=16)
    st = replay(sch, jobs)
    torch.cuda.synchronize()
    print(st.as_dict(), flush=True)
    assert st.n_jobs == len(jobs)
    assert max(sch.batch_sizes) > 1  # jobs were actually batched together
    for j in sorted(sch.done, key=lambda j: j.jid):
        # a batch sizes work items from its total work: alone and in the mix,
        # a job's sums are split differently, equal within rounding (1e-6 of
        # the peak, 10x inside the FP32 parity tolerance)
        alone = ism.simulate(j.room, j.src, j.rcv)
        torch.cuda.synchronize()
        peak = torch.amax(torch.abs(alone), dim=-1)
        err = torch.amax(torch.abs(alone - j.out), dim=-1)
        assert bool(torch.all(err <= 1e-6 * peak)), f"job {j.jid} differs alone vs in the mix"
