"""The allocation-free dense entry point (qsim_expect_circuit_noalloc) against
qsim_expect_circuit on the same inputs, through the C-ABI.

Two calls in a row share the GPU's fixed working memory, the second with a
smaller input (fewer qubits, a smaller batch, fewer slots and partial sums):
each must give the values of qsim_expect_circuit with its kept final states
bit for bit (the same plan and kernels), the final states in the caller's
buffer bit for bit, and the oracle's values within 1e-5 * sum|c| (complex64)
or 1e-10 * sum|c| (complex128).  Size errors come back from the host checks
before any device work.
"""
from __future__ import annotations

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Q():
    import paper_2112_10239_amd as Q

    return Q


def say(*a):
    print(*a, flush=True)


def _case(n, depth, batch, seed):
    c = W.brickwork_ry_rz_cnot(n, depth)
    H = W.tfim(n, 1.0)
    th = np.stack([W.angles(c.n_params, [seed, b, n]) for b in range(batch)])
    return c, H, th


def _check_pair(Q, ctx, oracle_mod, c, H, th, dtype, device_params=False):
    import torch

    rows = th.shape[0]
    cdt = torch.complex64 if dtype == Q.C64 else torch.complex128
    buf = torch.empty(rows * (1 << c.n), dtype=cdt, device="cuda:0")
    theta = torch.tensor(th, dtype=torch.float64, device="cuda:0") if device_params else th
    got = np.atleast_1d(ctx.expect_circuit_noalloc(c, H, theta, buf, dtype=dtype))
    want, kept = ctx.expect_circuit(c, H, th, mode=Q.MODE_DENSE, dtype=dtype, keep=True)
    want = np.atleast_1d(want)
    kept_psi = kept.to_host()
    kept.destroy()
    torch.cuda.synchronize()
    psi = buf.cpu().numpy().reshape(rows, 1 << c.n)
    assert np.array_equal(got, want), (got, want)
    assert np.array_equal(psi.view(np.uint8), kept_psi.view(np.uint8))
    tol = (1e-5 if dtype == Q.C64 else 1e-10) * H.abs_coeff_sum()
    for b in range(rows):
        ref = oracle_mod.expect(c, H, th[b])
        assert abs(got[b] - ref) <= tol, (b, got[b], ref)


def test_noalloc_two_calls_second_smaller(Q, oracle_mod):
    with Q.Context(0) as ctx:
        say("noalloc call 1: n=18 depth 6 batch 3 complex64")
        c, H, th = _case(18, 6, 3, 61)
        _check_pair(Q, ctx, oracle_mod, c, H, th, Q.C64)
        say("noalloc call 2: n=11 depth 3 batch 1 complex64")
        c, H, th = _case(11, 3, 1, 62)
        _check_pair(Q, ctx, oracle_mod, c, H, th, Q.C64)


def test_noalloc_complex128_and_device_params(Q, oracle_mod):
    with Q.Context(0) as ctx:
        say("noalloc complex128: n=14 depth 4 batch 2, then n=9 depth 2 batch 1")
        c, H, th = _case(14, 4, 2, 63)
        _check_pair(Q, ctx, oracle_mod, c, H, th, Q.C128)
        c, H, th = _case(9, 2, 1, 64)
        _check_pair(Q, ctx, oracle_mod, c, H, th, Q.C128)
        say("noalloc device parameters: n=16 depth 5 batch 2, then n=10 depth 2 batch 1")
        c, H, th = _case(16, 5, 2, 65)
        _check_pair(Q, ctx, oracle_mod, c, H, th, Q.C64, device_params=True)
        c, H, th = _case(10, 2, 1, 66)
        _check_pair(Q, ctx, oracle_mod, c, H, th, Q.C64, device_params=True)


def test_noalloc_size_errors(Q):
    import torch

    with Q.Context(0) as ctx:
        c, H, th = _case(10, 2, 1, 67)
        say("noalloc short state buffer")
        short = torch.empty((1 << 10) - 1, dtype=torch.complex64, device="cuda:0")
        with pytest.raises(Q.QsimError) as e:
            ctx.expect_circuit_noalloc(c, H, th[0], short)
        assert e.value.code == Q.qsim.EINVAL
        # n = 36: the partial sums alone take 2 * 2^23 * 8 B = 128 MiB (checked on the
        # host, before the state buffer and before any device work)
        say("noalloc working memory above the fixed maximum")
        c, H, th = _case(36, 1, 1, 68)
        with pytest.raises(Q.QsimError) as e:
            ctx.expect_circuit_noalloc(c, H, th[0], short)
        assert e.value.code == Q.qsim.ETOOBIG
        assert "fixed maximum" in str(e.value)
