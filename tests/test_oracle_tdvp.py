"""Pins of the oracle's 2TDVP (paper Section 2.1.2) against exact dynamics,
closed forms, invariants and library routines."""
import json
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import HBAR
from oracle import exact, tdvp
from oracle import hamiltonian as ham
from oracle import mpo as mpom
from oracle import mps as mpsm
from oracle import observables as obs
import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


# ---------------------------------------------------------------- Lanczos ----
def _rand_herm(rng, n):
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return (x + x.conj().T) / (2 * np.sqrt(n))


@pytest.mark.parametrize("n,tau", [(50, 0.3), (200, 1.0), (400, -0.7)])
def test_lanczos_matches_expm(n, tau):
    rng = np.random.default_rng(n)
    H = _rand_herm(rng, n)
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    y, it, ok = tdvp.lanczos_expm(lambda x: H @ x, v, tau)
    ref = scipy.linalg.expm(-1j * tau * H) @ v
    assert ok
    assert np.linalg.norm(y - ref) <= 1e-12 * np.linalg.norm(v)


def test_lanczos_unitarity_and_breakdown():
    rng = np.random.default_rng(7)
    H = _rand_herm(rng, 120)
    a = rng.standard_normal(120) + 1j * rng.standard_normal(120)
    b = rng.standard_normal(120) + 1j * rng.standard_normal(120)
    ya, _, _ = tdvp.lanczos_expm(lambda x: H @ x, a, 0.8)
    yb, _, _ = tdvp.lanczos_expm(lambda x: H @ x, b, 0.8)
    assert abs(np.vdot(ya, yb) - np.vdot(a, b)) < 1e-12 * np.linalg.norm(a) * np.linalg.norm(b)
    lam, Z = np.linalg.eigh(H)
    y, it, ok = tdvp.lanczos_expm(lambda x: H @ x, 3.0 * Z[:, 5], 0.8)
    assert it == 1 and ok  # exact invariant subspace: one application
    assert np.abs(y - 3.0 * np.exp(-0.8j * lam[5]) * Z[:, 5]).max() < 1e-13


def test_tridiag_expm_e1_vs_expm():
    rng = np.random.default_rng(3)
    a, b = rng.standard_normal(9), rng.random(8)
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    ref = scipy.linalg.expm(-0.4j * T)[:, 0]
    assert np.abs(tdvp.tridiag_expm_e1(a, b, 0.4) - ref).max() < 1e-14


# ------------------------------------------------------------ truncation ----
def test_choose_rank_rules():
    s = np.array([1.0, 0.5, 0.1, 1e-3, 1e-5, 1e-7])
    tot = np.sum(s ** 2)
    for eps in [1e-1, 1e-3, 1e-6, 1e-10, 1e-15]:
        k = tdvp.choose_rank(s, eps, 100)
        # brute force: smallest k with discarded weight <= eps * total
        ks = [j for j in range(1, len(s) + 1) if np.sum(s[j:] ** 2) <= eps * tot]
        assert k == min(ks)
    assert tdvp.choose_rank(s, 1e-15, 3) == 3
    assert tdvp.choose_rank(s, 1e-2, 100, sv_mode=1) == 3
    assert tdvp.choose_rank(s, 0.0, 4, sv_mode=2) == 4
    # a degenerate pair at the cut is kept whole
    s2 = np.array([1.0, 0.3, 0.3 * (1 - 1e-14), 0.01])
    assert tdvp.choose_rank(s2, 0.05, 100) == 3
    assert tdvp.choose_rank(np.array([1.0, 0.0, 0.0]), 0.0, 10) == 1


def test_svd_truncate_eckart_young():
    rng = np.random.default_rng(11)
    th = rng.standard_normal((6, 4, 3, 5)) + 1j * rng.standard_normal((6, 4, 3, 5))
    U, S, Vh, disc, s_all = tdvp.svd_truncate(th, 1e-2, 7)
    k = len(S)
    approx = np.einsum("ask,k,ktb->astb", U, S, Vh)
    assert abs(np.linalg.norm(th - approx) ** 2 - disc) < 1e-12 * np.linalg.norm(th) ** 2
    assert mpsm.left_orth_error(U) < 1e-13
    assert mpsm.right_orth_error(Vh) < 1e-13
    assert np.allclose(s_all, np.linalg.svd(th.reshape(24, 15), compute_uv=False), atol=1e-13)
    assert k <= 7


# ----------------------------------------------------- heff / environment ----
def test_heff2_spectrum_at_full_rank_crossover():
    """At a full-rank MPS every two-site H_eff is the full H in a complete
    basis: at the pair (1, 2) of config 1 (bonds 2 | 64) its spectrum is
    the spectrum of H."""
    model = synth.config1_model(0)
    model["nbasis"] = np.array([3, 3, 3, 3])
    dims = ham.site_dims(model)
    rng = np.random.default_rng(0)
    psi = rng.standard_normal(int(np.prod(dims))) + 0j
    psi /= np.linalg.norm(psi)
    st = tdvp.TDVP2(mpsm.from_dense_full_rank(psi, dims), mpom.build_mpo(model))
    # move the centre to site 1 by one exact left-orthonormalisation
    A0 = st.mps[0]
    q, r = np.linalg.qr(A0.reshape(-1, A0.shape[2]))
    st.mps[0] = q.reshape(A0.shape[0], A0.shape[1], -1)
    st.mps[1] = np.tensordot(r, st.mps[1], axes=([1], [0]))
    st.L[1] = tdvp.env_left(st.L[0], st.mps[0], st.W[0])
    st.R[3] = tdvp.env_right(tdvp.env_right(st.R[5], st.mps[4], st.W[4]), st.mps[3], st.W[3])
    Heff = tdvp.heff2_matrix(st.L[1], st.W[1], st.W[2], st.R[3])
    assert np.abs(Heff - Heff.conj().T).max() < 1e-13
    ev_eff = np.linalg.eigvalsh(Heff)
    ev_full = np.linalg.eigvalsh(ham.dense_hamiltonian(model).toarray())
    assert Heff.shape[0] == len(ev_full)
    assert np.abs(ev_eff - ev_full).max() < 1e-12
    # and the pairwise-contracted application agrees with the explicit matrix
    th = np.tensordot(st.mps[1], st.mps[2], axes=([2], [0]))
    assert np.abs(tdvp.heff2(st.L[1], st.W[1], st.W[2], st.R[3], th).reshape(-1)
                  - Heff @ th.reshape(-1)).max() < 1e-13


def test_heff_hermitian_random():
    p = synth.heff_problem(5, 4, 3, 2, 5, 3, 4, 2)
    H = tdvp.heff2_matrix(p["L"], p["W1"], p["W2"], p["R"])
    assert np.abs(H - H.conj().T).max() < 1e-14
    p1 = synth.heff_problem(6, 4, 3, 0, 5, 3, 0, 2, two_site=False)
    H1 = tdvp.heff1_matrix(p1["L"], p1["W"], p1["R"])
    assert np.abs(H1 - H1.conj().T).max() < 1e-14


# ----------------------------------------------------------- whole sweep ----
def _run(model, steps, D_max, eps, mps=None, sv_mode=0, dt=None):
    dims = ham.site_dims(model)
    W = mpom.build_mpo(model)
    psi = mps if mps is not None else mpsm.product_state(dims, model["occ"])
    st = tdvp.TDVP2(psi, W, sv_mode=sv_mode)
    dt = model["dt_fs"] if dt is None else dt
    disc = 0.0
    for _ in range(steps):
        disc += sum(st.step(dt, D_max, eps)["disc"])
    return st, disc


@pytest.mark.slow
def test_full_rank_exactness_config1():
    """With every bond at full rank and nothing truncated the tangent-space
    projector is the identity, so 2TDVP reproduces exp(-iHt)psi0."""
    model = synth.config1_model(0)
    dims = ham.site_dims(model)
    psi0 = exact.product_vector(model)
    full = mpsm.from_dense_full_rank(psi0, dims)
    assert mpsm.bond_dims(full) == [1, 2, 16, 64, 8, 1]
    st, _ = _run(model, 20, 64, 0.0, mps=full, sv_mode=2)
    ref = exact.evolve(model, psi0, [20 * model["dt_fs"]])[0]
    assert np.linalg.norm(mpsm.to_dense(st.mps) - ref) < 1e-10


def test_two_site_chain_is_exact():
    model = synth.config1_model(1)
    model = dict(model, omega=model["omega"][:1], nbasis=np.array([12]), g1=model["g1"][:1],
                 order=np.array([-1, 0]), occ=np.array([1, 0]))
    st, _ = _run(model, 5, 24, 0.0, sv_mode=2)
    ref = exact.evolve(model, exact.product_vector(model), [5 * model["dt_fs"]])[0]
    assert np.linalg.norm(mpsm.to_dense(st.mps) - ref) < 1e-12


def test_displaced_oscillator_autocorrelation():
    """No inter-state coupling: the state stays a product and C(t) has a
    closed form (sum over harmonic levels of a displaced oscillator)."""
    om, ka = np.array([0.12, 0.2]), np.array([0.09, -0.14])
    model = synth.single_mode_model(om, ka, nbasis=30, E=(0.3, -0.2), state=0)
    dims = ham.site_dims(model)
    psi0 = mpsm.product_state(dims, model["occ"])
    W = mpom.build_mpo(model)
    st = tdvp.TDVP2(psi0, W)
    for k in range(1, 9):
        st.step(0.5, 4, 1e-14)
        c = obs.overlap(psi0, st.mps)
        ref = exact.displaced_autocorrelation(0.5 * k, 0.3, om, ka)
        assert abs(c - ref) < 1e-12
    assert max(mpsm.bond_dims(st.mps)) == 1


def test_rabi_oscillation():
    model = synth.rabi_model(E0=0.0, E1=0.4, V01=0.05)
    st = tdvp.TDVP2(mpsm.product_state(ham.site_dims(model), model["occ"]),
                    mpom.build_mpo(model))
    for k in range(1, 11):
        st.step(0.5, 4, 1e-14)
        p = obs.populations(model, st.mps)
        assert abs(p[0] - exact.rabi_population(0.5 * k, 0.0, 0.4, 0.05)) < 1e-12


def test_sf_table1_electronic_dynamics():
    H = np.array(GOLD["sf_table1"]["H"])
    model = synth.sf_table1_model()
    assert np.allclose(np.diag(model["E"]) + model["V"], H, atol=0)
    st = tdvp.TDVP2(mpsm.product_state(ham.site_dims(model), model["occ"]),
                    mpom.build_mpo(model))
    for k in range(1, 11):
        st.step(0.5, 6, 1e-14)
        ref = exact.electronic_populations(H, 0, 0.5 * k)[0]
        assert np.abs(obs.populations(model, st.mps) - ref).max() < 1e-12


def test_norm_discarded_weight_and_energy():
    model = synth.config1_model(2)
    W = mpom.build_mpo(model)
    st, disc = _run(model, 6, 6, 1e-6)
    assert disc > 1e-8  # truncation actually happened
    assert abs(obs.norm2(st.mps) + disc - 1.0) < 1e-11
    # without truncation (full rank): norm and energy are conserved
    dims = ham.site_dims(model)
    psi0 = exact.product_vector(model)
    full = mpsm.from_dense_full_rank(psi0, dims)
    e0 = obs.energy(full, W)
    st2, _ = _run(model, 6, 64, 0.0, mps=full, sv_mode=2)
    assert abs(obs.norm2(st2.mps) - 1.0) < 1e-12
    assert abs(obs.energy(st2.mps, W) - e0) < 1e-10


def test_time_reversibility():
    model = synth.config1_model(4)
    model["nbasis"] = np.array([3, 3, 3, 3])
    dims = ham.site_dims(model)
    rng = np.random.default_rng(1)
    psi = rng.standard_normal(int(np.prod(dims))) + 1j * rng.standard_normal(int(np.prod(dims)))
    psi /= np.linalg.norm(psi)
    full = mpsm.from_dense_full_rank(psi, dims)
    st = tdvp.TDVP2(full, mpom.build_mpo(model), sv_mode=2)
    st.step(0.7, 100, 0.0)
    st.step(-0.7, 100, 0.0)
    assert np.linalg.norm(mpsm.to_dense(st.mps) - psi) < 1e-10


def test_observables_vs_dense():
    model = synth.config1_model(0)
    model["nbasis"] = np.array([3, 4, 3, 2])
    st, _ = _run(model, 3, 8, 1e-10)
    v = mpsm.to_dense(st.mps)
    H = ham.dense_hamiltonian(model)
    assert abs(obs.norm2(st.mps) - np.vdot(v, v).real) < 1e-13
    assert abs(obs.energy(st.mps, st.W) - np.vdot(v, H @ v).real) < 1e-13
    assert np.abs(obs.populations(model, st.mps) - exact.el_populations(model, v)).max() < 1e-13


def test_truncated_run_converges_to_exact():
    """Finite D_max: the population error against exact propagation does not
    grow as D_max increases (projection + truncation error only)."""
    model = synth.config1_model(0)
    psi0 = exact.product_vector(model)
    ref = exact.el_populations(model, exact.evolve(model, psi0, [5.0])[0])
    errs = []
    for D in [2, 4, 8, 16]:
        st, _ = _run(model, 10, D, 1e-14)
        errs.append(np.abs(obs.populations(model, st.mps) - ref).max())
    assert all(errs[k + 1] <= errs[k] * (1 + 1e-6) for k in range(3))
    assert errs[-1] < 1e-3


def test_debye_discretisation_sum_rule():
    """sum_I g_I^2 / (2 w_I) -> (1/pi) int J(w)/w dw = (2 lam/pi) atan(w_max/w_0)."""
    g = GOLD["debye"]
    limit = 2 * g["lambda"] / np.pi * np.arctan(g["omega_max"] / g["omega_0"])
    w, c = synth.debye_bath(40, g["lambda"], g["omega_0"], g["omega_max"])
    assert abs(np.sum(c ** 2 / (2 * w)) - 0.0716) < 5e-4
    w, c = synth.debye_bath(20000, g["lambda"], g["omega_0"], g["omega_max"])
    assert abs(np.sum(c ** 2 / (2 * w)) - limit) < 1e-5


def test_hbar_constant():
    assert HBAR == pytest.approx(0.6582119569, abs=0)


def test_heff2_block_against_brute_force():
    """heff2 and its one-block form equal the defining sum over every index
    (eq. two-site Hamiltonian), written out as plain loops on a tiny problem."""
    import itertools
    p = synth.heff_problem(21, 2, 3, 2, 3, 2, 3, 2)
    L, W1, W2, R, th = p["L"], p["W1"], p["W2"], p["R"], p["theta"]
    Dl, d1, d2, Dr = th.shape
    wl, wc, wr = L.shape[0], W1.shape[1], R.shape[0]
    full = tdvp.heff2(L, W1, W2, R, th)
    for a, b in [(0, 0), (1, 2)]:
        blk = tdvp.heff2_block(L, W1, W2, R, th, a, b)
        for s, t in itertools.product(range(d1), range(d2)):
            acc = 0j
            for w, x, y, A, S, Tt, B in itertools.product(range(wl), range(wc), range(wr), range(Dl),
                                                          range(d1), range(d2), range(Dr)):
                acc += L[w, a, A] * W1[w, x, s, S] * W2[x, y, t, Tt] * R[y, b, B] * th[A, S, Tt, B]
            assert abs(blk[s, t] - acc) < 1e-13
            assert abs(full[a, s, t, b] - acc) < 1e-13
