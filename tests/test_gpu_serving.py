"""GPU tests of the serving engine (dsmc_submit / dsmc_poll): jobs of mixed
N, d_x, K and models, submitted in waves while others run, give results equal
to dsmc_smooth alone, bit for bit; admission waits for free slots; a job that
can never fit fails cleanly."""
import time

import numpy as np
import pytest

from paper_2202_02264_amd import workloads as W

from parity import log, run_gpu

pytestmark = pytest.mark.gpu

FIELDS = ("traj", "logw", "log_Z", "status", "leaf_x", "leaf_logw", "leaf_logL", "ancestry",
          "logZ_inc", "row_lse", "index")


def _wait(G, srv, ids, timeout=120.0):
    t0 = time.time()
    pending = set(ids)
    codes = {}
    while pending and time.time() - t0 < timeout:
        for i in list(pending):
            rc, st = G.dsmc_poll(srv, i)
            if rc != G.DSMC_EAGAIN:
                codes[i] = rc
                pending.discard(i)
        time.sleep(0.002)
    assert not pending, f"jobs not finished: {sorted(pending)}"
    return codes


def test_served_jobs_equal_single_runs():
    import torch
    from paper_2202_02264_amd import dsmc as G
    jobs = [(W.sv(300, seed=1), 256, 11), (W.lg4d(77, seed=2), 128, 12), (W.sv(1, seed=3), 64, 13),
            (W.lg1d(513, seed=4), 256, 14), (W.sv(1000, seed=5), 1024, 15),
            (W.lg1d(2, seed=6), 256, 16), (W.sv(129, seed=7), 256, 17),
            (W.lg4d(40, seed=8), 128, 18), (W.lg1d(64, seed=9), 100, 19)]
    srv = G.Server(mem_budget=8 << 30, max_jobs=3, max_classes=6)
    models, outs, ids = [], [], []
    log("serving: submit wave 1")
    for k, (spec, N, seed) in enumerate(jobs):
        m = G.Model(spec)
        o = G.alloc_job_output(N, spec.d_x, spec.K, diagnostics=True)
        models.append(m)
        outs.append(o)
        ids.append(G.dsmc_submit(srv, m, N, seed, o))
        if k == 4:
            time.sleep(0.01)  # the rest arrive while the first wave runs
            log("serving: submit wave 2")
    codes = _wait(G, srv, ids)
    assert all(c == 0 for c in codes.values()), codes
    torch.cuda.synchronize()
    for (spec, N, seed), m, o, jid in zip(jobs, models, outs, ids):
        single = run_gpu(spec, N, seed, model=m)
        for f in FIELDS:
            np.testing.assert_array_equal(getattr(o, f).cpu().numpy(), single[f], err_msg=f"{spec.name} {f}")
        t_sub, t_start, t_done = G.dsmc_job_times(srv, jid)
        assert 0 < t_sub <= t_start <= t_done
    srv.close()


def test_job_too_large_fails_cleanly():
    from paper_2202_02264_amd import dsmc as G
    srv = G.Server(mem_budget=64 << 20, max_jobs=4, max_classes=1)
    spec = W.sv(3000, seed=1)
    m = G.Model(spec)
    o = G.alloc_job_output(1024, 1, spec.K)
    jid = G.dsmc_submit(srv, m, 1024, 1, o)
    codes = _wait(G, srv, [jid], timeout=30)
    assert codes[jid] == G.DSMC_ENOMEM
    small = W.sv(20, seed=2)
    m2 = G.Model(small)
    o2 = G.alloc_job_output(1024, 1, small.K)
    jid2 = G.dsmc_submit(srv, m2, 1024, 2, o2)
    codes = _wait(G, srv, [jid2], timeout=30)
    assert codes[jid2] == 0
    srv.close()


def test_cancel_and_admission_deadline():
    """One series slot per class: a long job occupies it, so jobs behind it stay
    queued.  A cancelled one fails with DSMC_ECANCELLED, one with a 1 ms
    admission deadline fails with DSMC_EDEADLINE, an unconstrained one runs
    after the first and equals dsmc_smooth alone; cancelling a running or
    finished job is refused with DSMC_EAGAIN."""
    from paper_2202_02264_amd import dsmc as G
    srv = G.Server(mem_budget=16 << 30, max_jobs=1, max_classes=2)
    big = W.sv(8192, seed=1)
    small = W.sv(50, seed=2)
    mb, ms = G.Model(big), G.Model(small)
    ob = G.alloc_job_output(4096, 1, big.K)
    oc = G.alloc_job_output(4096, 1, small.K)
    od = G.alloc_job_output(4096, 1, small.K)
    oe = G.alloc_job_output(4096, 1, small.K, diagnostics=True)
    log("serving: cancel / deadline")
    jb = G.dsmc_submit(srv, mb, 4096, 1, ob)
    jc = G.dsmc_submit(srv, ms, 4096, 2, oc)
    jd = G.dsmc_submit(srv, ms, 4096, 3, od, admit_deadline=0.001)
    je = G.dsmc_submit(srv, ms, 4096, 4, oe)
    assert G.dsmc_cancel(srv, jc) == G.DSMC_OK
    codes = _wait(G, srv, [jb, jc, jd, je])
    assert codes[jb] == 0
    assert codes[jc] == G.DSMC_ECANCELLED
    assert codes[jd] == G.DSMC_EDEADLINE
    assert codes[je] == 0
    assert G.dsmc_cancel(srv, je) == G.DSMC_EAGAIN
    single = run_gpu(small, 4096, 4, model=ms)
    np.testing.assert_array_equal(oe.traj.cpu().numpy(), single["traj"])
    srv.close()


def test_released_jobs_are_forgotten():
    """dsmc_job_release frees a finished job's record (its id becomes unknown);
    a job still queued or running is not released.  Many submit / poll /
    release cycles leave no record behind."""
    from paper_2202_02264_amd import dsmc as G
    srv = G.Server(mem_budget=4 << 30, max_jobs=8, max_classes=2)
    spec = W.sv(64, seed=3)
    m = G.Model(spec)
    outs = [G.alloc_job_output(256, 1, spec.K) for _ in range(16)]
    log("serving: release cycles")
    for wave in range(10):
        ids = [G.dsmc_submit(srv, m, 256, 100 * wave + k, outs[k]) for k in range(16)]
        codes = _wait(G, srv, ids)
        assert all(c == 0 for c in codes.values()), codes
        for i in ids:
            assert G.dsmc_job_release(srv, i) == G.DSMC_OK
            rc = G._lib.dsmc_poll(srv.handle, i, None)
            assert rc == G.DSMC_EINVAL
    big = W.sv(8192, seed=4)
    mb = G.Model(big)
    ob = G.alloc_job_output(4096, 1, big.K)
    jb = G.dsmc_submit(srv, mb, 4096, 1, ob)
    assert G.dsmc_job_release(srv, jb) == G.DSMC_EAGAIN  # queued or running
    _wait(G, srv, [jb])
    assert G.dsmc_job_release(srv, jb) == G.DSMC_OK
    srv.close()
