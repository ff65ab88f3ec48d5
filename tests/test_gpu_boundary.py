"""GPU checks of the boundary calls: per-term values and parameters resident in
device memory.

Per-term values <P_t> (coefficients not applied) are compared term by term
with the oracle's per-term values at 1e-5 (each |<P_t>| <= 1; complex64).
Parameters passed as device buffers must give the results of the same
parameters passed from the host, up to fp64 rounding of the device's
trigonometry (the coefficients are rounded to the state's precision in both
cases), and within the usual tolerance of the oracle.
"""
from __future__ import annotations

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


def oracle_terms(oracle_mod, c, H, th):
    psi = oracle_mod.statevector(c, th)
    _, re, im = oracle_mod.expect_state(c.n, psi, H)
    return re


# --- per-term values --------------------------------------------------------------------

@pytest.mark.parametrize("n,depth", [(12, 4), (20, 6), (21, 5)])
def test_terms_dense_tfim_family(Q, eng, oracle_mod, n, depth):
    c = W.brickwork_ry_rz_cnot(n, depth)
    H = W.tfim(n, 1.0)
    th = W.angles(c.n_params, [2, 1, n, depth])
    say("terms dense tfim", n, depth)
    got = eng.expect_terms(c, H, th, mode=Q.MODE_DENSE)
    want = oracle_terms(oracle_mod, c, H, th)
    np.testing.assert_allclose(got, want, atol=TOL64)
    # the weighted sum is the total
    assert abs(float(np.dot(H.coeff, got)) - eng.expect_circuit(c, H, th, mode=Q.MODE_DENSE)) <= tol(H)


def test_terms_random_paulis_all_modes(Q, eng, oracle_mod):
    rng = np.random.default_rng([50, 1])
    n = 13
    c = W.random_circuit(n, 80, rng, kinds=(W.RX, W.RY, W.RZ, W.CZ, W.CNOT, W.U1))
    th = W.angles(max(c.n_params, 1), [50, 2])[: c.n_params]
    H = W.random_hamiltonian(n, 12, rng, max_weight=3)
    H = W.Hamiltonian.from_terms(list(H.terms()) + [(0.5, [])])  # an identity term
    say("terms random, all modes")
    want = oracle_terms(oracle_mod, c, H, th)
    assert want[-1] == pytest.approx(1.0)
    for mode in (Q.MODE_DENSE, Q.MODE_LIGHTCONE, Q.MODE_LIGHTCONE_FACTORED):
        got = eng.expect_terms(c, H, th, mode=mode)
        np.testing.assert_allclose(got, want, atol=TOL64, err_msg=f"mode {mode}")
    # complex128 dense: per term to 1e-10
    np.testing.assert_allclose(eng.expect_terms(c, H, th, mode=Q.MODE_DENSE, dtype=Q.C128), want, atol=1e-10)


def test_terms_n500_both_cone_modes(Q, eng, oracle_mod):
    """The 750 MaxCut terms at n=500 one by one against the oracle's cones."""
    w = W.lightcone_maxcut()
    say("terms n500")
    _, want = oracle_mod.expect_lightcone(w.circuit, w.H, w.theta)
    for mode in (Q.MODE_LIGHTCONE, Q.MODE_LIGHTCONE_FACTORED):
        got = eng.expect_terms(w.circuit, w.H, w.theta, mode=mode)
        assert got.shape == (750,)
        np.testing.assert_allclose(got, want, atol=TOL64, err_msg=f"mode {mode}")


def test_terms_batched_rows(Q, eng, oracle_mod):
    w = W.batched_grad_tfim(batch=3, n=10, depth=3)
    got = eng.expect_terms(w.circuit, w.H, w.theta, mode=Q.MODE_DENSE)
    assert got.shape == (3, w.H.n_terms)
    for b in range(3):
        np.testing.assert_allclose(got[b], oracle_terms(oracle_mod, w.circuit, w.H, w.theta[b]), atol=TOL64)


# --- parameters in device memory --------------------------------------------------------

@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_device_coef_rows_equal_host_rows(Q, eng, dtype):
    """The coefficient rows built by the device kernel from device parameters equal,
    bit for bit, the rows the host builds (one fp64 definition serves both)."""
    import torch

    from tests.test_gpu_parity import _rotation_mix

    dt = Q.C64 if dtype == "c64" else Q.C128
    cases = [W.batched_grad_tfim(batch=3, n=14, depth=4), None]
    for k, w in enumerate(cases):
        if w is None:
            c, th = _rotation_mix(13, 5, 7)
            th = th[None, :]
        else:
            c, th = w.circuit, w.theta
        say("coef rows", dtype, k)
        host = eng.coef_rows(c, th, dtype=dt)
        dev = eng.coef_rows(c, torch.tensor(th, dtype=torch.float64, device="cuda:0"), dtype=dt)
        assert host.shape == dev.shape
        bad = np.nonzero(host != dev)
        assert bad[0].size == 0, f"case {k}: {bad[0].size} bytes differ, first at row/byte {bad[0][0]}/{bad[1][0]}"


def test_device_params_dense_and_grad(Q, eng, oracle_mod):
    import torch

    w = W.batched_grad_tfim(batch=4, n=14, depth=4)
    c, H = w.circuit, w.H
    say("device params dense + grad")
    th_dev = torch.tensor(w.theta, dtype=torch.float64, device="cuda:0")
    E_h = eng.expect_circuit(c, H, w.theta, mode=Q.MODE_DENSE)
    E_d = eng.expect_circuit(c, H, th_dev, mode=Q.MODE_DENSE)
    np.testing.assert_allclose(E_d, E_h, atol=1e-6)
    np.testing.assert_allclose(E_d, oracle_mod.expect(c, H, w.theta), atol=tol(H))
    Eg_h, g_h = eng.expect_grad(c, H, w.theta)
    Eg_d, g_d = eng.expect_grad(c, H, th_dev)
    np.testing.assert_allclose(g_d, g_h, atol=1e-6)
    np.testing.assert_allclose(Eg_d, Eg_h, atol=1e-6)
    psr = oracle_mod.grad_psr(c, H, w.theta[2])
    np.testing.assert_allclose(g_d[2], psr, atol=tol(H))
    # float32 device parameters are widened on the device
    E_f = eng.expect_circuit(c, H, th_dev.to(torch.float32), mode=Q.MODE_DENSE)
    np.testing.assert_allclose(E_f, oracle_mod.expect(c, H, w.theta.astype(np.float32).astype(np.float64)),
                               atol=tol(H))


def test_device_params_every_rotation_form(Q, eng, oracle_mod):
    """RX/RY/RZ/U1 and fixed angles with exact multiples of pi/2: factored blocks,
    product start and plain slots built on the device, amplitudes against the oracle."""
    import torch

    from tests.test_gpu_parity import _rotation_mix

    c, th = _rotation_mix(13, 5, 7)
    say("device params rotation forms")
    psi_o = oracle_mod.statevector(c, th)
    st = eng.create_state(13, batch=1, dtype=Q.C64)
    st.apply_layer(c.gates, torch.tensor(th[None, :], dtype=torch.float64, device="cuda:0"), c.n_params,
                   mats=c.mats)
    psi = st.to_host()[0]
    st.destroy()
    np.testing.assert_allclose(psi, psi_o, atol=2e-6)
    # complex128 with device parameters
    st = eng.create_state(13, batch=1, dtype=Q.C128)
    st.apply_layer(c.gates, torch.tensor(th[None, :], dtype=torch.float64, device="cuda:0"), c.n_params,
                   mats=c.mats)
    np.testing.assert_allclose(st.to_host()[0], psi_o, atol=1e-12)
    st.destroy()


def test_device_params_mixed_layers(Q, eng, oracle_mod):
    """Layers with host and device parameters queued on one state."""
    import torch

    n, depth, B = 10, 4, 3
    c = W.brickwork_ry_rz_cnot(n, depth)
    H = W.tfim(n, 0.5)
    th = np.stack([W.angles(c.n_params, [51, b]) for b in range(B)])
    st = eng.create_state(n, batch=B)
    per_layer = len(c.gates) // depth
    ppl = c.n_params // depth
    for layer in range(depth):
        g = c.gates[layer * per_layer:(layer + 1) * per_layer].copy()
        g["param"] = np.where(g["param"] >= 0, g["param"] - layer * ppl, -1)
        p = th[:, layer * ppl:(layer + 1) * ppl]
        if layer % 2:
            p = torch.tensor(p, dtype=torch.float64, device="cuda:0")
        st.apply_layer(g, p, ppl)
    np.testing.assert_allclose(st.expect(H), oracle_mod.expect(c, H, th), atol=tol(H))
    st.destroy()


def test_device_params_cones(Q, eng, oracle_mod):
    import torch

    w = W.lightcone_maxcut(n=60, depth=3)
    th_dev = torch.tensor(w.theta, dtype=torch.float64, device="cuda:0")
    say("device params cones")
    want, _ = oracle_mod.expect_lightcone(w.circuit, w.H, w.theta)
    for mode in (Q.MODE_LIGHTCONE, Q.MODE_LIGHTCONE_FACTORED):
        assert abs(eng.expect_circuit(w.circuit, w.H, th_dev, mode=mode) - want) <= tol(w.H)
        E_h, g_h = eng.expect_grad(w.circuit, w.H, w.theta, mode=mode)
        E_d, g_d = eng.expect_grad(w.circuit, w.H, th_dev, mode=mode)
        np.testing.assert_allclose(g_d, g_h, atol=1e-6)
        assert abs(E_d - E_h) <= 1e-6


def test_autograd_device_theta(Q, eng, oracle_mod):
    """The autograd Function with theta on the device (never copied to the host)."""
    import torch

    from paper_2112_10239_amd.autograd import expectation

    w = W.batched_grad_tfim(batch=2, n=10, depth=3)
    theta = torch.tensor(w.theta, dtype=torch.float64, device="cuda:0", requires_grad=True)
    say("autograd device theta")
    E = expectation(theta, eng, w.circuit, w.H)
    assert E.is_cuda
    (E * torch.tensor([1.5, -1.0], dtype=torch.float64, device="cuda:0")).sum().backward()
    for row, wt in enumerate((1.5, -1.0)):
        psr = oracle_mod.grad_psr(w.circuit, w.H, w.theta[row])
        np.testing.assert_allclose(theta.grad[row].cpu().numpy(), wt * psr, atol=2 * tol(w.H))
