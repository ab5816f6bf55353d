"""Every output at the full benchmark sizes, against the fast CPU reference
(oracle/fast: Algorithms 1 and 2 and the spectral routes of Sections 3.2 and
4 in float64, pinned to the oracle's definitions in tests/test_oracle_fast.py).

  * p = 2, m = 24, s = 20 (the headline step's shape and inputs): all 2^24
    forward coefficients of the device-sampled exponential family, the
    integer transform bit for bit, the ANOVA variances at every d and the
    effective dimensions, and the interpolant at random 32-digit queries;
  * p = 3, m = 14, s = 10 (the interpolation workload): all forward
    coefficients, the inverse of arbitrary complex data, the variances, and
    the interpolant at random 20-digit queries;
  * the 512-job ragged batch: every coefficient of every job, grouped static
    passes and the one-launch schedule.

Tolerances: float32 data and float32 transforms carry a few float32
roundings per value (relative ~1e-7 normwise over m stages); 1e-5 is the
float bar used throughout (normwise, and max-abs relative to the largest
value).  The variances are float64 sums over float32 spectra of the data:
relative 1e-5 of the total variance per d.  Integer transforms (mod 2^32)
are exact.
"""
import numpy as np
import pytest
import torch

from oracle import anova, fast
from paper_0808_0487_amd import fdwt, inputs
from tests.gpu_common import announce, nrel

pytestmark = pytest.mark.gpu


def qdev(Q):
    return torch.from_numpy(np.ascontiguousarray(Q, dtype=np.int64).astype(np.uint32).view(np.int32)).cuda()


def close(got, ref, tol=1e-5):
    assert nrel(got, ref) <= tol, nrel(got, ref)
    assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref))


def dims_agree(res, vt, vs):
    """Effective dimensions equal, unless the reference's variance at the
    deciding d lies within the tolerance of the 0.99 threshold."""
    dt, ds = anova.effective_dims(vt, vs)
    tot = vt[-1]
    for got, want, v in ((res["d_trc"], dt, vt), (res["d_sup"], ds, vs)):
        if got != want:
            near = [abs(v[d] - 0.99 * tot) <= 1e-5 * tot for d in (got, want)]
            assert any(near), (got, want)


@pytest.mark.timeout(600)
def test_headline_step_every_output():
    p, m, s = 2, 24, 20
    announce("full step vs fast reference", p, m, s)
    C = inputs.upper_triangular_generators(p, m, s, seed=2)
    a = inputs.family_params("exp", s, ratio=0.1)
    gam = inputs.kernel_weights(s)
    X = fast.net_int(p, m, C)
    ref_ft = fast.fwt(p, m, fast.sample("exp", p, m, a, X))
    net = fdwt.Net(p, m, s, C)
    kern = fdwt.Kernel(2.0, gam)
    ft = net.forward_family("exp", a)
    close(ft.cpu().numpy().astype(np.float64), ref_ft)
    # integer data: the unnormalised transform mod 2^32, bit for bit
    fi = inputs.uniform_int32(p ** m, -1000, 1000, seed=3)
    gi = net.forward(torch.from_numpy(fi).cuda()).cpu().numpy()
    exact = np.rint(fast.fwt(p, m, fi.astype(np.float64)) * p ** m).astype(np.int64)
    assert np.array_equal(gi, (exact & 0xFFFFFFFF).astype(np.uint32).view(np.int32))
    # ANOVA variances at every d
    res = net.eff_dim(kern, ft)
    vt, vs = fast.variances(p, m, 2.0, gam, X, ref_ft)
    tot = vt[-1]
    assert np.max(np.abs(res["var_trc"] - vt)) <= 1e-5 * tot
    assert np.max(np.abs(res["var_sup"] - vs)) <= 1e-5 * tot
    dims_agree(res, vt, vs)
    # interpolant at random queries and at net points
    D = inputs.QUERY_DEPTH[p]
    Q = inputs.queries(p, s, 24, 11).astype(np.int64)
    idx = [0, 5, p ** m - 1]
    Qall = np.concatenate([Q, X[:, idx] * p ** (D - m)], axis=1)
    f = net.sample("exp", a)
    _, sf = net.walsh_interp(kern, f, qdev(Qall))
    c_ref = fast.spline_coef(p, m, 2.0, gam, X, ref_ft)
    ref_sf = fast.spline_eval(p, m, 2.0, gam, X, c_ref, Qall, D)
    close(sf.cpu().numpy().astype(np.float64), ref_sf)
    net.close()


@pytest.mark.timeout(600)
def test_interpolation_workload_every_output():
    p, m, s = 3, 14, 10
    announce("full p3 vs fast reference", p, m, s)
    C = inputs.upper_triangular_generators(p, m, s, seed=3)
    a = inputs.family_params("product", s, alpha=2.0)
    gam = inputs.kernel_weights(s)
    X = fast.net_int(p, m, C)
    ref_f = fast.sample("product", p, m, a, X)
    ref_ft = fast.fwt(p, m, ref_f)
    net = fdwt.Net(p, m, s, C)
    kern = fdwt.Kernel(2.0, gam)
    f = net.sample("product", a)
    close(f.cpu().numpy().astype(np.float64), ref_f)
    ft = net.forward(f)
    close(ft.cpu().numpy().astype(np.complex128), ref_ft)
    # inverse of arbitrary complex data (no Hermitian symmetry)
    g = np.random.default_rng(21)
    ct = (g.standard_normal(p ** m) + 1j * g.standard_normal(p ** m)).astype(np.complex64)
    back = net.inverse(torch.from_numpy(ct).cuda()).cpu().numpy().astype(np.complex128)
    close(back, fast.fwt(p, m, ct.astype(np.complex128), inverse=True))
    # variances
    res = net.eff_dim(kern, ft)
    vt, vs = fast.variances(p, m, 2.0, gam, X, ref_ft)
    tot = vt[-1]
    assert np.max(np.abs(res["var_trc"] - vt)) <= 1e-5 * tot
    assert np.max(np.abs(res["var_sup"] - vs)) <= 1e-5 * tot
    dims_agree(res, vt, vs)
    # interpolant at random 20-digit queries and at net points
    D = inputs.QUERY_DEPTH[p]
    Q = inputs.queries(p, s, 48, 12).astype(np.int64)
    idx = [0, 77, p ** m - 1]
    Qall = np.concatenate([Q, X[:, idx] * p ** (D - m)], axis=1)
    _, sf = net.walsh_interp(kern, f, qdev(Qall))
    c_ref = fast.spline_coef(p, m, 2.0, gam, X, ref_ft)
    ref_sf = fast.spline_eval(p, m, 2.0, gam, X, c_ref, Qall, D)
    close(sf.cpu().numpy().astype(np.float64), ref_sf)
    net.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", ["f32", "f32_one_launch"])
def test_batch_workload_every_coefficient(prec):
    """The benchmark's 512 jobs (m in 12..22), uniform data, every output."""
    announce("full batch vs fast reference", prec)
    specs = inputs.batch_jobs(512, seed=4)
    jobs = []
    for i, (m, s, alpha, cseed) in enumerate(specs):
        x = torch.from_numpy(inputs.uniform_float(2 ** m, 7000 + i)).cuda()
        jobs.append((m, x, torch.empty_like(x)))
    b = fdwt.Batch(jobs, precision=prec)
    b.run()
    b.check()
    for i, (m, x, y) in enumerate(jobs):
        ref = fast.fwt(2, m, x.cpu().numpy().astype(np.float64))
        got = y.cpu().numpy().astype(np.float64)
        assert nrel(got, ref) <= 1e-5, (i, m)
        assert np.max(np.abs(got - ref)) <= 1e-5 * np.max(np.abs(ref)), (i, m)
    b.close()
