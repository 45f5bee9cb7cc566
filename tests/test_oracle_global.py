"""Pins of the oracle's global integrators (paper Section 2.1.1: RK4 and
the global Krylov method) against dense linear algebra: the MPO x MPS
product against H psi, sums against vector sums, compression without
truncation against the identity, RK4 against the 4th-order Taylor
polynomial of the propagator, global Krylov against exact propagation."""
import numpy as np
import pytest
import scipy.linalg

from oracle import HBAR, exact
from oracle import globalprop as gp
from oracle import hamiltonian as ham
from oracle import mpo as mpom
from oracle import mps as mpsm
from oracle import tdvp
import synth


def _state(seed=0, steps=2, D=6):
    model = synth.config1_model(seed)
    model["nbasis"] = np.array([3, 3, 3, 3])
    W = mpom.build_mpo(model)
    st = tdvp.TDVP2(mpsm.product_state(ham.site_dims(model), model["occ"]), W)
    for _ in range(steps):
        st.step(1.0, D, 1e-12)
    return model, W, st.mps


def test_apply_mpo_and_lincomb_are_dense_operations():
    model, W, psi = _state()
    H = ham.dense_hamiltonian(model).toarray()
    v = mpsm.to_dense(psi)
    assert np.abs(mpsm.to_dense(gp.apply_mpo(W, psi)) - H @ v).max() < 1e-13
    _, _, phi = _state(1, 3, 4)
    s = gp.lincomb([0.3 - 0.2j, 1.7], [psi, phi])
    assert np.abs(mpsm.to_dense(s) - ((0.3 - 0.2j) * v + 1.7 * mpsm.to_dense(phi))).max() < 1e-14


def test_compress_without_truncation_is_exact_and_canonical():
    model, W, psi = _state()
    x = gp.apply_mpo(W, psi)
    y, disc = gp.compress(x, 10 ** 6, 0.0, sv_mode=2)
    assert np.abs(mpsm.to_dense(y) - mpsm.to_dense(x)).max() < 1e-12
    assert disc < 1e-24
    for a in y[1:]:
        assert mpsm.right_orth_error(a) < 1e-12
    assert max(mpsm.bond_dims(y)) <= max(mpsm.full_rank_caps(ham.site_dims(model)))


def test_rk4_is_the_fourth_order_taylor_polynomial():
    """For a time-independent H the RK4 update equals sum_{k<=4} (-i H dt/hbar)^k / k! psi."""
    model, W, psi = _state()
    H = ham.dense_hamiltonian(model).toarray()
    v = mpsm.to_dense(psi)
    dt = 0.4
    A = -1j * dt / HBAR * H
    ref = v.copy()
    term = v.copy()
    for k in range(1, 5):
        term = A @ term / k
        ref = ref + term
    got = gp.rk4_step(psi, W, dt, 10 ** 6, 1e-15)
    assert np.linalg.norm(mpsm.to_dense(got) - ref) < 1e-11
    # and it is not the exact propagator (fifth-order error is visible)
    exact_v = scipy.linalg.expm(A) @ v
    assert np.linalg.norm(ref - exact_v) > 1e-8


def test_taylor2_norm_growth_closed_form():
    """U_2 = 1 - i tau H - tau^2 H^2 / 2 gives U_2^H U_2 = 1 + tau^4 H^4 / 4,
    so without truncation |psi'|^2 = |psi|^2 + tau^4 |H^2 psi|^2 / 4: the
    second-order method the paper runs does not conserve the norm."""
    model, W, psi = _state()
    H = ham.dense_hamiltonian(model).toarray()
    v = mpsm.to_dense(psi)
    dt = 0.6
    tau = dt / HBAR
    got = mpsm.to_dense(gp.taylor_step(psi, W, dt, 10 ** 6, 0.0, order=2))
    want = np.vdot(v, v).real + tau ** 4 * np.linalg.norm(H @ (H @ v)) ** 2 / 4
    assert abs(np.vdot(got, got).real - want) < 1e-12 * want
    assert want - np.vdot(v, v).real > 1e-8  # the growth is visible


def test_taylor_high_order_is_the_exact_propagator():
    model, W, psi = _state()
    H = ham.dense_hamiltonian(model).toarray()
    v = mpsm.to_dense(psi)
    got = gp.taylor_step(psi, W, 0.4, 10 ** 6, 0.0, order=25)
    ref = scipy.linalg.expm(-1j * 0.4 / HBAR * H) @ v
    assert np.linalg.norm(mpsm.to_dense(got) - ref) < 1e-11


def test_global_krylov_matches_exact_propagation():
    model, W, psi = _state()
    H = ham.dense_hamiltonian(model).toarray()
    v = mpsm.to_dense(psi)
    got, m = gp.global_krylov_step(psi, W, 0.8, 10 ** 6, 1e-15, m_max=20, tol=1e-12)
    ref = scipy.linalg.expm(-1j * 0.8 / HBAR * H) @ v
    assert np.linalg.norm(mpsm.to_dense(got) - ref) < 1e-10
    assert 3 <= m < 20


def test_global_krylov_grows_bonds_from_a_single_excitation():
    """The paper's use: global steps from the product state |S2> x |0> in the
    per-state chain, where two-site steps alone cannot start the inter-state
    coupling (three sites apart); the result follows exact propagation."""
    m = synth.lvc4_per_state_model(0, "default")
    m["nbasis"] = np.array([4, 3, 3, 4])
    W = mpom.build_mpo(m)
    psi0 = mpsm.product_state(ham.site_dims(m), m["occ"])
    x = psi0
    for _ in range(3):
        x, _ = gp.global_krylov_step(x, W, m["dt_fs"], 64, 1e-14, m_max=16, tol=1e-11)
    assert max(mpsm.bond_dims(x)) > 1
    ref = exact.evolve(m, exact.product_vector(m), [3 * m["dt_fs"]])[0]
    # every compression drops a relative weight <= 1e-14 per bond
    assert np.linalg.norm(mpsm.to_dense(x) - ref) < 1e-6


def _random_full_rank(model, seed):
    dims = ham.site_dims(model)
    rng = np.random.default_rng(seed)
    v = rng.normal(size=int(np.prod(dims))) + 1j * rng.normal(size=int(np.prod(dims)))
    return mpsm.from_dense_full_rank(v / np.linalg.norm(v), dims)


def test_variational_apply_exact_without_truncation():
    """eq. variational app with bonds at full rank and nothing truncated:
    the fitted |phi> is H|psi> itself (dense H built element by element)."""
    model, _, _ = _state()
    W = mpom.build_mpo(model)
    psi = _random_full_rank(model, 1)
    H = ham.dense_hamiltonian(model).toarray()
    phi, sweeps = gp.apply_mpo_variational(W, psi, 10 ** 6, 0.0)
    assert np.abs(mpsm.to_dense(phi) - H @ mpsm.to_dense(psi)).max() < 1e-12
    assert sweeps <= 5  # settles to the rounding level of the norm within a few sweeps
    for A in phi[1:]:
        assert mpsm.right_orth_error(A) < 1e-12


def test_variational_apply_two_sites_is_eckart_young():
    """On a two-site chain the variational minimum of eq. variational app at
    rank k is the rank-k SVD truncation of H|psi> (Eckart-Young)."""
    model = synth.rabi_model(E0=0.0, E1=0.4, V01=0.05)
    model["omega"] = np.array([0.1])
    model["nbasis"] = np.array([6])
    model["g1"] = np.array([[[0.05, 0.02], [0.02, -0.04]]])
    W = mpom.build_mpo(model)
    dims = ham.site_dims(model)
    psi = _random_full_rank(model, 2)
    H = ham.dense_hamiltonian(model).toarray()
    hv = (H @ mpsm.to_dense(psi)).reshape(dims[0], dims[1])
    u, s, vh = np.linalg.svd(hv)
    ref = (u[:, :1] * s[:1]) @ vh[:1]
    phi, _ = gp.apply_mpo_variational(W, psi, 1, 0.0)
    assert np.abs(mpsm.to_dense(phi).reshape(dims[0], dims[1]) - ref).max() < 1e-12


def test_variational_apply_truncated_is_optimal_projection():
    """With bonds capped, the fitted |phi> is stationary (<phi|H psi> =
    <phi|phi>, the projection property of the minimum) and no farther from
    H|psi> than the direct route's compression at the same bonds."""
    model, _, _ = _state()
    W = mpom.build_mpo(model)
    psi = _random_full_rank(model, 3)
    H = ham.dense_hamiltonian(model).toarray()
    hv = H @ mpsm.to_dense(psi)
    for D in (3, 5, 8):
        phi, _ = gp.apply_mpo_variational(W, psi, D, 0.0, sweeps=20, tol=1e-15)
        f = mpsm.to_dense(phi)
        assert abs(np.vdot(f, hv) - np.vdot(f, f)) < 1e-10 * np.vdot(f, f).real
        direct, _ = gp.compress(gp.apply_mpo(W, psi), D, 0.0)
        assert np.linalg.norm(f - hv) <= np.linalg.norm(mpsm.to_dense(direct) - hv) * (1 + 1e-9)
        assert max(mpsm.bond_dims(phi)) <= D


def test_global_krylov_variational_apply_is_exact_propagation():
    """The global Krylov step with the variational MPO application at full
    rank is exact propagation, as with the direct product."""
    model, W, psi = _state()
    H = ham.dense_hamiltonian(model).toarray()
    dt = 0.6
    out, _ = gp.global_krylov_step(psi, W, dt, 10 ** 6, 0.0, m_max=24, tol=1e-12, apply="variational")
    ref = scipy.linalg.expm(-1j * dt / HBAR * H) @ mpsm.to_dense(psi)
    assert np.abs(mpsm.to_dense(out) - ref).max() < 1e-10
