"""Ragged batches of p = 2 transforms (grouped static passes, the generic
persistent launch per pass level with float32 or bfloat16-split low stages,
and every pass of every job in one persistent launch), against the oracle,
alone vs in the mix, tuned, and under HIP-graph capture."""
import numpy as np
import pytest
import torch

from oracle import walsh
from paper_0808_0487_amd import fdwt, inputs
from tests.gpu_common import announce, nrel, sample_indices

pytestmark = pytest.mark.gpu


def make_jobs(ms, seed):
    jobs = []
    for i, m in enumerate(ms):
        x = torch.from_numpy(inputs.uniform_float(2 ** m, seed + i)).cuda()
        jobs.append((m, x, torch.empty_like(x)))
    return jobs


def check_against_oracle(jobs, tol, seed):
    for i, (m, x, y) in enumerate(jobs):
        f = x.cpu().numpy().astype(np.float64)
        hs = sample_indices(2 ** m, 64, seed + i)
        err = nrel(y.cpu().numpy()[hs], walsh.dwt_phase(2, m, f, hs))
        assert err <= tol, (i, m, err)


MS = [7, 9, 12, 13, 14, 15, 17, 20, 22, 8, 16, 19, 21, 13, 10, 3, 1, 6, 23]


@pytest.mark.parametrize("prec,tol", [("f32", 1e-5), ("f32_generic", 1e-5), ("bf16x2", 2e-5), ("f32_one_launch", 1e-5)])
def test_ragged_batch_against_oracle(prec, tol):
    announce("batch", prec)
    jobs = make_jobs(MS, 500)
    b = fdwt.Batch(jobs, precision=prec)
    b.run()
    b.check()
    check_against_oracle(jobs, tol, 500)
    b.close()


def test_one_launch_repeatable_and_in_place():
    """Every pass of every job in one launch (ticket order, per-job pass
    counters, static 2^13-element tiles for m >= 13): the oracle's values,
    and the same bits on consecutive runs (counters reset per run) and with
    the jobs in place."""
    announce("batch one launch")
    ms = MS + [18, 18, 11, 24]
    jobs = make_jobs(ms, 1000)
    b = fdwt.Batch(jobs, "f32_one_launch")
    b.run()
    b.check()
    check_against_oracle(jobs[:-1], 1e-5, 1000)
    first = [y.clone() for _, _, y in jobs]
    for rep in range(3):
        for _, _, y in jobs:
            y.fill_(float(rep))
        b.run()
        b.check()
        for i, ((_, _, y), r) in enumerate(zip(jobs, first)):
            assert torch.equal(y, r), (rep, i)
    b.close()
    inplace = [(m, x.clone()) for m, x, _ in jobs[:6]]
    ip = fdwt.Batch([(m, x, x) for m, x in inplace], "f32_one_launch")
    ip.run()
    ip.check()
    for (m, x), r in zip(inplace, first[:6]):
        assert torch.equal(x, r), m
    ip.close()


def test_one_launch_at_the_largest_sizes():
    """Jobs of 2^24..2^26 points (three passes: waits on the first and the
    second pass) beside tiny ones, against the oracle at sampled outputs."""
    announce("batch one launch max sizes")
    ms = [26, 1, 25, 2, 24, 13]
    jobs = make_jobs(ms, 1200)
    b = fdwt.Batch(jobs, "f32_one_launch")
    b.run()
    b.check()
    for i, (m, x, y) in enumerate(jobs):
        f = x.cpu().numpy().astype(np.float64)
        hs = sample_indices(2 ** m, 6 if m > 20 else 64, 1200 + i)
        assert nrel(y.cpu().numpy()[hs], walsh.dwt_phase(2, m, f, hs)) <= 1e-5, m
    b.close()


def test_one_launch_wait_failure_is_reported(monkeypatch):
    """With the wait limit set to zero on the host every dependency wait gives
    up: each workgroup leaves the launch, the launch ends, and check reports
    FDWT_ETIMEOUT; a batch created without the setting then runs normally."""
    announce("batch one launch forced give-up")
    jobs = make_jobs([18, 20, 12], 1300)
    monkeypatch.setenv("FDWT_BATCH_WAIT_MS", "0")
    b = fdwt.Batch(jobs, "f32_one_launch")
    monkeypatch.delenv("FDWT_BATCH_WAIT_MS")
    b.run()
    with pytest.raises(fdwt.FdwtError) as ei:
        b.check()
    assert ei.value.code == fdwt.ETIMEOUT
    b.close()
    ok = fdwt.Batch(jobs, "f32_one_launch")
    ok.run()
    ok.check()
    check_against_oracle(jobs, 1e-5, 1300)
    ok.close()


def test_one_launch_graph_replays_match_eager():
    announce("batch one launch graph")
    jobs = make_jobs([12, 16, 19, 9], 1100)
    b = fdwt.Batch(jobs, "f32_one_launch")
    b.run()
    b.check()
    eager = [y.clone() for _, _, y in jobs]
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        b.run(stream=s)
    for rep in range(3):
        for _, _, y in jobs:
            y.fill_(float(rep + 1))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        b.check()
        for e, (_, _, y) in zip(eager, jobs):
            assert torch.equal(e, y), rep


def test_bf16_split_error_is_reported_scale():
    """The two-term bfloat16 split represents x to about 2^-18; the batched
    result stays within 1e-5 normwise of the float64 transform, and differs
    from the float32 path by more than float32 rounding (the MFMA path ran)."""
    announce("bf16 split error")
    m = 16
    jobs32 = make_jobs([m], 900)
    jobs16 = [(m, jobs32[0][1], torch.empty_like(jobs32[0][1]))]
    fdwt.Batch(jobs32, "f32").run()
    fdwt.Batch(jobs16, "bf16x2").run()
    torch.cuda.synchronize()
    f = jobs32[0][1].cpu().numpy().astype(np.float64)
    ref = np.fft.fftn(f.reshape([2] * m, order="F")).reshape(2 ** m, order="F").real / 2 ** m
    e32 = nrel(jobs32[0][2].cpu().numpy(), ref)
    e16 = nrel(jobs16[0][2].cpu().numpy(), ref)
    assert e32 <= 1e-6 and e16 <= 1e-5 and e16 > 2 * e32, (e32, e16)


def test_alone_equals_in_the_mix_bit_identical():
    announce("batch alone vs mix")
    jobs = make_jobs(MS, 600)
    fdwt.Batch(jobs, "f32").run()
    torch.cuda.synchronize()
    for i in [0, 3, 8, 12]:
        m, x, y = jobs[i]
        z = torch.empty_like(x)
        fdwt.Batch([(m, x, z)], "f32").run()
        torch.cuda.synchronize()
        assert torch.equal(y, z), i


def test_in_place_and_against_single_transform():
    announce("batch in place")
    m = 18
    x = torch.from_numpy(inputs.uniform_float(2 ** m, 7)).cuda()
    y = x.clone()
    fdwt.Batch([(m, y, y)], "f32").run()
    net = fdwt.Net(2, m, 1, inputs.identity_generators(2, m, 1))
    ref = net.forward(x)
    torch.cuda.synchronize()
    assert float(torch.linalg.norm(y - ref) / torch.linalg.norm(ref)) <= 1e-6


def test_graph_capture_replays_match_eager():
    announce("batch graph capture")
    jobs = make_jobs([12, 16, 19], 700)
    b = fdwt.Batch(jobs, "f32")
    b.run()
    torch.cuda.synchronize()
    eager = [y.clone() for _, _, y in jobs]
    for _, _, y in jobs:
        y.zero_()
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        b.run(stream=s)
    for rep in range(3):
        for _, _, y in jobs:
            y.fill_(float(rep + 1))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for e, (_, _, y) in zip(eager, jobs):
            assert torch.equal(e, y), rep
    b.check()


def test_autotune_keeps_results_exact():
    """The tuner times every distinct plan per group and keeps one; results
    after tuning still match the oracle, and the chosen plans are reported."""
    announce("batch autotune")
    ms = [12, 12, 15, 18, 18, 21, 22]
    jobs = make_jobs(ms, 800)
    b = fdwt.Batch(jobs, "f32")
    b.autotune(reps=3)
    for _, _, y in jobs:
        y.fill_(0.0)
    b.run()
    b.check()
    check_against_oracle(jobs, 1e-5, 800)
    groups = b.describe()
    assert sorted(g[0] for g in groups) == sorted(set(ms))
    assert all(10 <= g[1] <= 14 for g in groups)
    assert sum(g[2] for g in groups) == len(ms)
    b.close()


def test_batch_rejects_bad_jobs():
    x = torch.empty(16, device="cuda")
    with pytest.raises(ValueError):
        fdwt.Batch([(5, x, x)])
    with pytest.raises(KeyError):
        fdwt.Batch([(4, x, x)], precision="fp8")
