"""GPU parity of the dense pass under every per-context tile shape, through the
C-ABI: tile qubits m in 12..14, register bits r in 3..5 (r >= m - 10, at most
1024 threads per workgroup), always-local low bits 4 or 6, and the factored
rotations, folds and register prefetch switched off one at a time.  Each
context evaluates the same seeded circuits as the default context and is
compared with the oracle at 1e-5 * sum|c| (complex64).

n = 21 with m = 12 runs 512 tiles per row, n = 23 more tiles than resident
workgroups (the persistent walk with a non-zero stride at every tile shape).
"""
from __future__ import annotations

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-5

SHAPES = [(12, 3), (12, 4), (12, 5), (13, 3), (13, 4), (13, 5), (14, 4), (14, 5)]


@pytest.fixture(scope="module")
def Q():
    import paper_2112_10239_amd as Q

    return Q


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def cases(oracle_mod):
    out = []
    for n, depth in ((17, 8), (21, 5), (23, 3)):
        c = W.brickwork_ry_rz_cnot(n, depth)
        H = W.tfim(n, 1.0)
        th = W.angles(c.n_params, [31, n, depth])
        out.append((n, depth, c, H, th, oracle_mod.expect(c, H, th)))
    rng = np.random.default_rng(32)
    c = W.random_circuit(18, 150, rng)
    H = W.random_hamiltonian(18, 16, rng, max_weight=4)
    th = W.angles(max(c.n_params, 1), [32, 1])[: c.n_params]
    out.append((18, 0, c, H, th, oracle_mod.expect(c, H, th)))
    return out


def _check(Q, ctx, cases, label):
    for n, depth, c, H, th, want in cases:
        say(label, "n", n, "depth", depth)
        got = ctx.expect_circuit(c, H, th, mode=Q.MODE_DENSE)
        assert abs(got - want) <= TOL64 * max(1.0, H.abs_coeff_sum()), (label, n, depth, got, want)
        again = ctx.expect_circuit(c, H, th, mode=Q.MODE_DENSE)
        assert again == got, (label, n, "repeat differs")


@pytest.mark.parametrize("m,r", SHAPES)
@pytest.mark.parametrize("clow", [4, 6])
def test_tile_shapes_vs_oracle(Q, cases, m, r, clow):
    ctx = Q.Context(0, tile_qubits=m, register_bits=r, coalesce_bits=clow)
    try:
        _check(Q, ctx, cases, f"m={m} r={r} clow={clow}")
    finally:
        ctx.close()


@pytest.mark.parametrize("off", ["OFF_FACTORED", "OFF_ABSORB", "OFF_ENTRY", "OFF_EXIT", "OFF_PRODUCT",
                                 "OFF_PREFETCH", "OFF_IO_REGS", "OFF_RELABEL", "OFF_EARLY_TERMS"])
def test_switches_vs_oracle(Q, cases, off):
    import paper_2112_10239_amd.qsim as qs

    for m, r in ((13, 4), (13, 5)):
        ctx = Q.Context(0, tile_qubits=m, register_bits=r, disable=getattr(qs, off))
        try:
            _check(Q, ctx, cases, f"{off} m={m} r={r}")
        finally:
            ctx.close()
