"""GPU parity on the launch shapes the full-size workloads take.

The dense n=30 workload walks several tiles per persistent workgroup and has
two measurement passes; the batched gradient workload builds its coefficient
rows on several host threads; the serving stream mixes requests of up to 28
qubits and depth 16; some plans store a tile in its first stage through a
permutation.  Each of these paths is checked here against the oracle at sizes
the oracle still finishes in seconds, with the same launch code as the
full-size runs.  Tolerances as in test_gpu_parity: complex64 results within
1e-5 * sum|coeff| of the complex128 oracle.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-5


@pytest.fixture(scope="module")
def Q():
    import paper_2112_10239_amd as Q

    return Q


@pytest.fixture(scope="module")
def eng(Q):
    ctx = Q.Context(0)
    yield ctx
    ctx.close()


def tol(H):
    return TOL64 * max(1.0, H.abs_coeff_sum())


def say(*a):
    print(*a, flush=True)


def ring_zz(n):
    return W.Hamiltonian.from_terms([(1.0, [(i, "Z"), ((i + 1) % n, "Z")]) for i in range(n)])


# --- the dense family at the sizes where the tile walk and the plan shapes change -----

@pytest.mark.parametrize("n,depth,fixed", [(23, 20, False), (24, 20, False), (24, 20, True)])
def test_dense_tfim_full_paths(Q, eng, oracle_mod, n, depth, fixed):
    """n=23: each resident workgroup walks more than one tile (non-zero stride);
    n=24: the relabelled plan with X terms measured in the gate passes and one
    measurement pass, and (fixed) the plan that keeps every qubit at its own
    index bit and measures X terms at the end (two measurement passes).  A second
    call on the same inputs gives the same bits (fixed reduction order).  Every
    term's value <P_t> is checked too, at 1e-5 each (the 2n TFIM terms have unit
    weight), so one wrong term cannot hide in the sum."""
    import paper_2112_10239_amd.qsim as qs

    c = W.brickwork_ry_rz_cnot(n, depth)
    H = W.tfim(n, 1.0)
    th = W.angles(c.n_params, [2, 1, n, depth])
    ctx = Q.Context(0, disable=qs.OFF_RELABEL | qs.OFF_EARLY_TERMS) if fixed else eng
    try:
        ps = ctx.plan_passes(c, H)
        meas_only = sum(1 for p in ps if p["flags"] == 66)
        early = sum(1 for p in ps if p["flags"] & 64 and p["flags"] & 4)
        say("dense tfim full paths", n, depth, "fixed" if fixed else "relabel", len(ps), "passes", meas_only,
            "measurement passes", early, "storing passes that measure")
        if n == 24:
            assert meas_only == (2 if fixed else 1)
            assert fixed or early >= 2
        psi = oracle_mod.statevector(c, th)
        want, want_terms, _ = oracle_mod.expect_state(c.n, psi, H)
        del psi
        got = ctx.expect_circuit(c, H, th, mode=Q.MODE_DENSE)
        assert abs(got - want) <= tol(H), (got, want)
        again = ctx.expect_circuit(c, H, th, mode=Q.MODE_DENSE)
        assert again == got
        got_terms = ctx.expect_terms(c, H, th, mode=Q.MODE_DENSE)
        np.testing.assert_allclose(got_terms, want_terms, rtol=0, atol=TOL64)
    finally:
        if fixed:
            ctx.close()


# --- passes that store in their first stage through a permutation -----------------------

def test_store_first_stage_tfim_n15(Q, eng, oracle_mod):
    """Kept final state with X terms measured at the end (the plan keeps every
    qubit at its own index bit and has the shape); the default expectation runs
    the relabelled plan with X terms measured in the gate passes."""
    import paper_2112_10239_amd.qsim as qs

    c = W.brickwork_ry_rz_cnot(15, 9)
    H = W.tfim(15, 1.0)
    th = W.angles(c.n_params, [40, 15, 9])
    say("store-first-stage tfim n15 d9")
    want = oracle_mod.expect(c, H, th)
    fixed = Q.Context(0, disable=qs.OFF_EARLY_TERMS | qs.OFF_RELABEL)
    try:
        got, st = fixed.expect_circuit(c, H, th, mode=Q.MODE_DENSE, keep=True)
        st.destroy()
    finally:
        fixed.close()
    assert abs(got - want) <= tol(H), (got, want)
    again = eng.expect_circuit(c, H, th, mode=Q.MODE_DENSE)
    assert abs(again - want) <= tol(H), (again, want)


@pytest.mark.parametrize("fixed", [True, False])
def test_store_first_stage_zz_keep_and_grad(Q, eng, oracle_mod, fixed):
    """CNOT brickwork n=14 depth 2 with a ZZ-only H: with qubits kept at their own
    index bits (fixed) the kept (stored) final state gets its measurement in a stage
    after the storing one; by default the kept plan relabels and its last pass puts
    the qubits back in order (the kept state is compared amplitude by amplitude)."""
    import paper_2112_10239_amd.qsim as qs

    n = 14
    c = W.brickwork_ry_rz_cnot(n, 2)
    H = ring_zz(n)
    th = W.angles(c.n_params, [41, n])
    say("store-first-stage zz keep n14 d2", "fixed" if fixed else "relabelled")
    want = oracle_mod.expect(c, H, th)
    ctx = Q.Context(0, disable=qs.OFF_EARLY_TERMS | qs.OFF_RELABEL) if fixed else eng
    try:
        E, st = ctx.expect_circuit(c, H, th, mode=Q.MODE_DENSE, keep=True)
        assert abs(E - want) <= tol(H), (E, want)
        psi = st.to_host()[0]
        st.destroy()
        np.testing.assert_allclose(psi, oracle_mod.statevector(c, th), atol=2e-6)
        E2, g = ctx.expect_grad(c, H, th)
        assert abs(E2 - want) <= tol(H)
        np.testing.assert_allclose(g, oracle_mod.grad_psr(c, H, th), atol=tol(H))
    finally:
        if fixed:
            ctx.close()


def test_kept_state_relabelled_vs_oracle(Q, eng, oracle_mod):
    """Kept states of relabelled plans at n = 16, 18 and 20 (a pass of its own puts the
    qubits back in order at n = 20): every amplitude against the oracle's."""
    for n, depth in ((16, 8), (18, 6), (20, 10)):
        c = W.brickwork_ry_rz_cnot(n, depth)
        H = W.tfim(n, 0.5)
        th = W.angles(c.n_params, [42, n, depth])
        say("kept relabelled", n, depth, len(eng.plan_passes(c, H, keep=True)), "passes")
        E, st = eng.expect_circuit(c, H, th, mode=Q.MODE_DENSE, keep=True)
        psi = st.to_host()[0]
        st.destroy()
        assert abs(E - oracle_mod.expect(c, H, th)) <= tol(H)
        np.testing.assert_allclose(psi, oracle_mod.statevector(c, th), atol=2e-6)


# --- the batched gradient workload at its own batch --------------------------------------

def test_grad_tfim_b256(Q, eng, oracle_mod):
    """B=256 rows (the host builds coefficient rows on several threads): E of every
    fourth row against the oracle, shift-rule entries of rows 0, 1, 127 and 255."""
    w = W.batched_grad_tfim(batch=256)
    c, H = w.circuit, w.H
    say("grad tfim b256")
    E, g = eng.expect_grad(c, H, w.theta)
    rows = np.unique(np.concatenate([np.arange(0, 256, 4), [1, 127, 255]]))
    want = oracle_mod.expect(c, H, w.theta[rows])
    np.testing.assert_allclose(E[rows], want, atol=tol(H))
    rng = np.random.default_rng([4, 9])
    for row in (0, 1, 127, 255):
        idx = np.sort(rng.choice(c.n_params, size=8, replace=False)).astype(np.int32)
        psr = oracle_mod.grad_psr(c, H, w.theta[row], idx)
        np.testing.assert_allclose(g[row, idx], psr, atol=tol(H))


# --- serving at the large end of the request mix --------------------------------------

def _run_all(eng, reqs):
    tickets = [(r, eng.submit(r.circuit, r.H, r.theta, r.want_grad)) for r in reqs]
    res = {}
    pending = dict((t, r) for r, t in tickets)
    while pending:
        for t, r in list(pending.items()):
            st, E, g = eng.poll(t, r.circuit.n_params)
            if st == 1:
                continue
            assert st == 0, st
            res[r.rid] = (E, g)
            del pending[t]
    return res


def test_serving_mix_large(Q, eng, oracle_mod):
    """Requests of 20-24 qubits at depth 16 (half with gradients): each result alone
    equals its value in the mix bit for bit, and matches the oracle."""
    reqs = [W.serving_request(1000 + r, n_range=(20, 24), depth_range=(16, 16)) for r in range(10)]
    say("serving mix large", [(r.n, r.want_grad) for r in reqs])
    alone = {}
    for r in reqs[:4]:
        alone.update(_run_all(eng, [r]))
    mix = _run_all(eng, reqs)
    for rid, (E, g) in alone.items():
        assert mix[rid][0] == E
        if g is not None:
            np.testing.assert_array_equal(mix[rid][1], g)
    for r in reqs[:6]:
        want = oracle_mod.expect(r.circuit, r.H, r.theta)
        assert abs(mix[r.rid][0] - want) <= tol(r.H), (r.rid, mix[r.rid][0], want)
        if r.want_grad and r.n <= 22:
            idx = np.arange(0, r.circuit.n_params, max(1, r.circuit.n_params // 4), dtype=np.int32)
            psr = oracle_mod.grad_psr(r.circuit, r.H, r.theta, idx)
            np.testing.assert_allclose(mix[r.rid][1][idx], psr, atol=tol(r.H))
