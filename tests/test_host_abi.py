"""Host-side checks of libqsim that need no GPU: exported symbols, light-cone
sets, plan validity and the serving scheduler on a host-only context (the
executor is simulated: every launch completes at once and computes nothing)."""
from __future__ import annotations

import os
import re
import subprocess
import sys
import time

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def Q():
    lib = os.path.join(ROOT, "paper_2112_10239_amd", "libqsim.so")
    if not os.path.exists(lib):
        from paper_2112_10239_amd import build as b

        b.build()
    import paper_2112_10239_amd as Q

    return Q


def header_functions():
    with open(os.path.join(ROOT, "include", "qsim.h")) as f:
        src = f.read()
    return sorted(set(re.findall(r"\b(qsim_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol(Q):
    names = header_functions()
    assert len(names) >= 18
    out = subprocess.run(["nm", "-D", "--defined-only", Q.qsim.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (qsim_[a-z0-9_]+)$", out, re.M))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    assert set(Q.qsim.EXPORTS) == set(names)


def test_lightcone_sets_bit_exact(Q, oracle_mod):
    w = W.lightcone_maxcut()
    a = Q.lightcone_sets(w.circuit, w.H)
    b = oracle_mod.lightcone_sets(w.circuit, w.H)
    assert len(a) == len(b) == 750
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    for seed in range(5):
        rng = np.random.default_rng([30, seed])
        n = int(rng.integers(3, 40))
        c = W.random_circuit(n, 80, rng)
        H = W.random_hamiltonian(n, 15, rng, max_weight=3)
        assert all(np.array_equal(x, y) for x, y in zip(Q.lightcone_sets(c, H), oracle_mod.lightcone_sets(c, H)))


def check_plan_order(c, order):
    """Every gate exactly once; on every qubit, gates run in circuit order."""
    assert sorted(order[:, 3].tolist()) == list(range(c.n_gates))
    pos = {int(g): (int(p), int(s), int(o)) for p, s, o, g in order}
    last = {}
    for g, row in enumerate(c.gates):
        qs = [int(row["q0"])] + ([int(row["q1"])] if int(row["kind"]) in W.TWO_QUBIT else [])
        for q in qs:
            if q in last:
                a, b = pos[last[q]], pos[g]
                assert a < b or (a == b and last[q] < g), (q, last[q], g, a, b)
            last[q] = g


@pytest.mark.parametrize("make", [lambda: W.dense_tfim().circuit, lambda: W.small_ring_maxcut().circuit,
                                  lambda: W.batched_grad_tfim(batch=1).circuit, lambda: W.brickwork_ry_cz(28, 16)])
def test_plan_valid_named(Q, make):
    c = make()
    info, order = Q.plan_dense(c)
    check_plan_order(c, order)
    assert info["passes"] >= 1


@pytest.mark.parametrize("seed", range(6))
def test_plan_valid_random(Q, seed):
    rng = np.random.default_rng([31, seed])
    n = int(rng.integers(1, 34))
    c = W.random_circuit(n, 300, rng)
    info, order = Q.plan_dense(c)
    check_plan_order(c, order)


def test_dense_plan_pass_count(Q):
    """The n=30 depth-20 brickwork needs far fewer passes than one per gate layer and qubit block:
    15 with relabelled passes and X terms measured in the gate passes (24 without either)."""
    info, _ = Q.plan_dense(W.dense_tfim().circuit, W.dense_tfim().H)
    assert info["passes"] <= 16 and info["meas_passes"] <= 1, info


# --- serving scheduler on a host-only context ------------------------------------------

def wait(ctx, t, n_params=0, timeout=20.0):
    t0 = time.time()
    while True:
        st, E, g = ctx.poll(t, n_params)
        if st != 1:
            return st, E, g
        if time.time() - t0 > timeout:
            raise TimeoutError(t)
        time.sleep(0.001)


def test_serving_mock_lifecycle(Q):
    ctx = Q.Context(-1, hbm_budget_bytes=1 << 30, max_queue=64)
    reqs = [W.serving_request(r, n_range=(12, 20), depth_range=(4, 8)) for r in range(20)]
    tickets = [ctx.submit(r.circuit, r.H, r.theta, r.want_grad) for r in reqs]
    assert len(set(tickets)) == len(tickets)
    for r, t in zip(reqs, tickets):
        st, E, g = wait(ctx, t, r.circuit.n_params if r.want_grad else 0)
        assert st == 0
        assert E >= 1  # the simulated executor reports the number of passes it ran
        if r.want_grad:
            assert g.shape == (r.circuit.n_params,)
    # a consumed ticket is gone
    assert ctx.poll(tickets[0])[0] == Q.qsim.ENOTFOUND
    s = ctx.server_stats()
    assert s["completed"] == 20 and s["inflight_bytes"] == 0 and s["running"] == 0
    assert 0 < s["peak_inflight_bytes"] <= 1 << 30
    ctx.close()


def test_serving_mock_budget_and_queue(Q):
    ctx = Q.Context(-1, hbm_budget_bytes=64 << 20, max_queue=4)
    big = W.serving_request(0, n_range=(25, 25))
    with pytest.raises(Q.QsimError) as ei:  # 2^25 * 8 B = 256 MiB > 64 MiB budget
        ctx.submit(big.circuit, big.H, big.theta, False)
    assert ei.value.code == Q.qsim.ETOOBIG
    small = [W.serving_request(r, n_range=(12, 12), depth_range=(16, 16)) for r in range(12)]
    got, rejected = [], 0
    for r in small:
        try:
            got.append(ctx.submit(r.circuit, r.H, r.theta, False))
        except Q.QsimError as e:
            assert e.code == Q.qsim.EAGAIN
            rejected += 1
    assert got
    for t in got:
        assert wait(ctx, t)[0] == 0
    assert ctx.server_stats()["rejected"] == rejected + 1
    ctx.close()


def test_serving_mock_cancel_and_shutdown(Q, monkeypatch):
    # simulated steps of 20 ms: the last of ten requests is still queued when it is cancelled
    monkeypatch.setenv("QSIM_TEST_MOCK_STEP_MS", "20")
    ctx = Q.Context(-1, hbm_budget_bytes=(1 << 24) + (1 << 22), max_queue=100)
    reqs = [W.serving_request(r, n_range=(20, 20), depth_range=(16, 16)) for r in range(10)]
    ts = [ctx.submit(r.circuit, r.H, r.theta, True) for r in reqs]
    assert ctx.cancel(ts[-1]) == 0
    assert wait(ctx, ts[-1])[0] == Q.qsim.ECANCELED
    assert ctx.cancel(123456789) == Q.qsim.ENOTFOUND
    ctx.close()  # remaining tickets end with ESHUTDOWN; nothing leaks or hangs


def test_serving_mock_alloc_failure_isolated():
    """An allocation failure (forced by the test hook) fails one request; the others complete."""
    code = r"""
import sys, time
sys.path.insert(0, %r)
import paper_2112_10239_amd as Q, workloads as W
ctx = Q.Context(-1, hbm_budget_bytes=1 << 34)
reqs = [W.serving_request(r, n_range=(12, 14), depth_range=(4, 6)) for r in range(6)]
ts = [ctx.submit(r.circuit, r.H, r.theta, False) for r in reqs]
res = []
for t in ts:
    while True:
        st = ctx.poll(t)[0]
        if st != 1:
            break
        time.sleep(0.001)
    res.append(st)
print(res)
ctx.close()
""" % ROOT
    env = dict(os.environ, QSIM_TEST_FAIL_ALLOC="3")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=120)
    assert out.returncode == 0, out.stderr
    res = eval(out.stdout.strip().splitlines()[-1])
    assert res.count(-2) == 1 and res.count(0) == 5


def test_serving_mock_accounting_covers_pool(Q, monkeypatch):
    """In-flight accounting is at least the device bytes the pool hands out (every block of
    every admitted request: states, plan descriptors, coefficients, partial sums, results)."""
    monkeypatch.setenv("QSIM_TEST_MOCK_STEP_MS", "1")
    budget = 3 << 24
    ctx = Q.Context(-1, hbm_budget_bytes=budget, max_queue=200)
    reqs = [W.serving_request(r, n_range=(14, 21), depth_range=(4, 12)) for r in range(40)]
    ts = [ctx.submit(r.circuit, r.H, r.theta, r.want_grad) for r in reqs]
    seen_out = 0
    for t in ts:
        while True:
            s = ctx.server_stats()
            assert s["pool_outstanding_bytes"] <= s["inflight_bytes"] <= budget
            seen_out = max(seen_out, s["pool_outstanding_bytes"])
            st = ctx.poll(t)[0]
            if st != 1:
                break
            time.sleep(0.0005)
        assert st == 0
    s = ctx.server_stats()
    assert s["accounting_violations"] == 0 and seen_out > 0
    assert s["inflight_bytes"] == 0 and s["pool_outstanding_bytes"] == 0
    assert s["peak_inflight_bytes"] <= budget
    ctx.close()


def test_serving_poll_sizes_gradient_buffer(Q):
    """Polling a gradient request without stating n_params still returns the whole gradient (regression:
    the binding used to hand the library a one-element buffer)."""
    ctx = Q.Context(-1, hbm_budget_bytes=1 << 32)
    r = W.serving_request(3, n_range=(14, 14), depth_range=(10, 10))
    t = ctx.submit(r.circuit, r.H, r.theta, True)
    st, E, g = wait(ctx, t)
    assert st == 0 and g is not None and g.shape == (r.circuit.n_params,)
    ctx.close()


def test_plan_passes_store_first_stage_shapes(Q):
    """Plans with a pass that stores in its first stage through a permutation and
    measures in later stages (the loads of every wave must finish before any wave
    stores): the dense n=30 workload, and the shapes the GPU parity tests run."""
    import paper_2112_10239_amd.qsim as qs

    ctx = Q.Context(-1)
    # the shape is that of plans that keep qubits at their own index bits and measure X terms at the end
    fixed = Q.Context(-1, disable=qs.OFF_EARLY_TERMS | qs.OFF_RELABEL)
    try:
        def hazards(c, H, keep=False):
            ps = (fixed if keep else ctx).plan_passes(c, H, keep=keep)
            return [p for p in ps if p["store_stage"] == 0 and (p["entry_perm"] or p["exit_perm"])
                    and p["stages"] > 1]

        # (plans that keep the final state, X terms at the end: expectation-only plans relabel qubits)
        w = W.dense_tfim()
        assert hazards(w.circuit, w.H, keep=True)
        assert hazards(W.brickwork_ry_rz_cnot(15, 9), W.tfim(15, 1.0), keep=True)
        assert hazards(W.brickwork_ry_rz_cnot(23, 20), W.tfim(23, 1.0), keep=True)
        zz = W.Hamiltonian.from_terms([(1.0, [(i, "Z"), ((i + 1) % 14, "Z")]) for i in range(14)])
        assert hazards(W.brickwork_ry_rz_cnot(14, 2), zz, keep=True)
        # every pass record is consistent with its flags
        for p in ctx.plan_passes(w.circuit, w.H):
            assert p["stages"] >= 1 and p["m"] == 13
            assert (p["store_stage"] >= 0) == bool(p["flags"] & 4)
            assert (p["meas_index"] >= 0) == bool(p["flags"] & 64)
    finally:
        ctx.close()
        fixed.close()



def test_marshalling_cache_follows_edits():
    """The C views kept on circuits and Hamiltonians are reused only while they still
    describe the object: an in-place gate edit, a replaced array or U1 matrices give a
    fresh view; a Hamiltonian view points into its arrays, so edits in place are seen."""
    from paper_2112_10239_amd import qsim as qs

    w = W.small_ring_maxcut()
    c = w.circuit
    a = qs.CCircuit.of(c)
    assert qs.CCircuit.of(c) is a
    c.gates["q0"][0] = (c.gates["q0"][0] + 1) % c.n
    b = qs.CCircuit.of(c)
    assert b is not a and b._rec["q0"][0] == c.gates["q0"][0]
    c.gates = c.gates.copy()
    assert qs.CCircuit.of(c) is not b
    bld = W.GateListBuilder(2)
    bld.custom(0, np.eye(2))
    u = bld.build()
    assert qs.CCircuit.of(u) is not qs.CCircuit.of(u)  # U1 matrices: never cached
    H = w.H
    h = qs.CHamiltonian.of(H)
    assert qs.CHamiltonian.of(H) is h
    H.coeff[0] = 7.0
    assert h.h.coeff[0] == 7.0  # the view points into the live array
    H.coeff = H.coeff.copy()
    assert qs.CHamiltonian.of(H) is not h
