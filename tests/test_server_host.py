"""Host-side sizing and validation of serving requests (no device)."""
import numpy as np
import pytest

from paper_0808_0487_amd import fdwt, inputs


def req(kind, p, m, s, nq=64, seed=1):
    C = inputs.upper_triangular_generators(p, m, s, seed)
    q = inputs.queries(p, s, nq, seed) if kind == "interp" else None
    return fdwt.Request(kind, p, m, s, C, seed, "product", inputs.family_params("product", s, alpha=2.0), 2.0,
                        inputs.kernel_weights(s), q)


@pytest.mark.parametrize("p,m,s", [(2, 10, 4), (2, 20, 30), (3, 9, 5), (5, 6, 7)])
def test_request_bytes_cover_buffers_and_caches(p, m, s):
    """Interpolation: the job holds f, the coefficients, c, queries and Sf;
    the caches are the float64 spectrum (N doubles, complex for p odd) and
    the packed coordinates (s N words, 4 or 8 bytes).  Effective dimension:
    the only cache is the spectrum."""
    N = p ** m
    jb, cb = fdwt.request_bytes(req("interp", p, m, s))
    spec = N * (8 if p == 2 else 16)
    packed = s * N * (4 if p == 2 else 8)
    assert cb >= spec + packed and cb <= spec + packed + 1024
    assert jb >= N * 4 + N * (4 if p == 2 else 8) + N * 4 + s * 64 * 4 + 64 * 4
    je, ce = fdwt.request_bytes(req("eff_dim", p, m, s))
    assert spec <= ce <= spec + 512
    # eff_dim holds at least one kernel-data column (8 B) and its transform
    assert je >= N * 4 + N * 8 + N * (8 if p == 2 else 16)


def test_effdim_chunk_bounds_job_memory():
    r = req("eff_dim", 2, 20, 30)
    small, _ = fdwt.request_bytes(r, effdim_chunk_bytes=1 << 20)
    large, _ = fdwt.request_bytes(r, effdim_chunk_bytes=8 << 30)
    N = 2 ** 20
    # one column per chunk vs all 2s = 60 columns, 16 B each
    assert large - small >= 59 * N * 16
    assert small < 8 * N * 16


def test_request_validation_on_host():
    r = req("interp", 2, 8, 3)
    r.p = 11
    with pytest.raises(fdwt.FdwtError) as e:
        fdwt.request_bytes(r)
    assert e.value.code == fdwt.EUNSUPPORTED
    r = req("interp", 2, 8, 3)
    r.alpha = 1.0
    with pytest.raises(fdwt.FdwtError):
        fdwt.request_bytes(r)
    r = req("interp", 3, 8, 3)
    r.C[0, 0, 0] = 3
    with pytest.raises(fdwt.FdwtError):
        fdwt.request_bytes(r)
    with pytest.raises(ValueError):
        fdwt.Request("interp", 2, 4, 2, np.zeros((2, 4, 4), np.uint8), 1, "exp", np.ones(2), 2.0, np.ones(2))


def test_arena_allocator_against_byte_map(tmp_path):
    """The server's device-arena bookkeeping (best fit, coalescing, exact
    accounting), compiled for the host and checked against a byte map over
    200000 random allocations and releases."""
    import os
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    exe = str(tmp_path / "arena_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", os.path.join(root, "paper_0808_0487_amd", "csrc"),
                    os.path.join(root, "tests", "arena_check.cpp"), "-o", exe], check=True, timeout=120)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout
