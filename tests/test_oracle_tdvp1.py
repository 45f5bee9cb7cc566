"""Pins of the oracle's one-site TDVP (paper Section 2.1.2, the 1TDVP scheme
with eq. zero-site Hamiltonian) against exact dynamics, closed forms, the
dense definition of the projected Hamiltonians and the invariants the paper
states for the scheme (norm and energy conserved, bond dimensions fixed)."""
import numpy as np

from oracle import exact, tdvp
from oracle import hamiltonian as ham
from oracle import mpo as mpom
from oracle import mps as mpsm
from oracle import observables as obs
import synth


def _small_config1(seed, nbasis=(3, 3, 3, 3)):
    model = synth.config1_model(seed)
    model["nbasis"] = np.array(nbasis)
    return model


def _grown(model, steps, D_max, dt=None):
    """A state with non-trivial, non-full bonds: a few two-site steps from the
    initial product state (no truncation below 1e-12 of the weight)."""
    W = mpom.build_mpo(model)
    st = tdvp.TDVP2(mpsm.product_state(ham.site_dims(model), model["occ"]), W)
    for _ in range(steps):
        st.step(model["dt_fs"] if dt is None else dt, D_max, 1e-12)
    return st.mps, W


def _block_bases(mps, b):
    """Dense left block basis (sites < b, columns = bond index) and right
    block basis (sites >= b, rows = bond index) of a mixed-canonical MPS
    whose sites < b are left- and sites >= b right-orthonormal."""
    left = np.ones((1, 1), dtype=complex)
    for a in mps[:b]:
        left = np.tensordot(left, a, axes=([1], [0])).reshape(-1, a.shape[2])
    right = np.ones((1, 1), dtype=complex)
    for a in reversed(mps[b:]):
        right = np.tensordot(a, right, axes=([2], [0])).reshape(a.shape[0], -1)
    return left, right


def test_splits_are_orthonormal_factorisations():
    rng = np.random.default_rng(0)
    M = rng.standard_normal((6, 3, 9)) + 1j * rng.standard_normal((6, 3, 9))
    A, C = tdvp.split_left(M)
    assert mpsm.left_orth_error(A) < 1e-14
    assert np.abs(np.tensordot(A, C, axes=([2], [0])) - M).max() < 1e-13
    C, B = tdvp.split_right(M)
    assert mpsm.right_orth_error(B) < 1e-14
    assert np.abs(np.tensordot(C, B, axes=([1], [0])) - M).max() < 1e-13


def test_heff0_is_the_projected_hamiltonian():
    """H_eff,0 at bond b equals <L_a R_b| H |L_a' R_b'> formed from the dense
    Hamiltonian and the dense block bases (eq. zero-site Hamiltonian)."""
    model = _small_config1(3)
    mps, W = _grown(model, 2, 5)
    H = ham.dense_hamiltonian(model)
    st = tdvp.TDVP1(mps, W)
    n = st.n
    # move the centre to bond b by left-orthonormalising sites < b
    b = 2
    for i in range(b):
        st.mps[i], C = tdvp.split_left(st.mps[i])
        st.L[i + 1] = tdvp.env_left(st.L[i], st.mps[i], W[i])
        st.mps[i + 1] = np.tensordot(C, st.mps[i + 1], axes=([1], [0]))
    # the bond matrix sits between sites b-1 and b: split it off site b
    C, st.mps[b] = tdvp.split_right(st.mps[b])
    st.R[b] = tdvp.env_right(st.R[b + 1], st.mps[b], W[b])
    left, right = _block_bases(st.mps, b)
    basis = np.einsum("xa,by->xyab", left, right).reshape(H.shape[0], -1)
    ref = basis.conj().T @ H @ basis
    got = tdvp.heff0_matrix(st.L[b], st.R[b])
    assert ref.shape == got.shape and ref.shape[0] > 4
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
    # and the apply agrees with the matrix
    rng = np.random.default_rng(1)
    x = rng.standard_normal(C.shape) + 1j * rng.standard_normal(C.shape)
    assert np.abs(tdvp.heff0(st.L[b], st.R[b], x).reshape(-1) - got @ x.reshape(-1)).max() < 1e-12
    assert n == 5


def test_full_rank_exactness():
    """Every bond at full rank: both projectors of the splitting are the
    identity, all terms equal H and commute, so 1TDVP is exact."""
    model = _small_config1(0)
    dims = ham.site_dims(model)
    psi0 = exact.product_vector(model)
    full = mpsm.from_dense_full_rank(psi0, dims)
    W = mpom.build_mpo(model)
    st = tdvp.TDVP1(full, W)
    for _ in range(6):
        assert st.step(model["dt_fs"])["converged"]
    ref = exact.evolve(model, psi0, [6 * model["dt_fs"]])[0]
    assert np.linalg.norm(mpsm.to_dense(st.mps) - ref) < 1e-10
    assert mpsm.bond_dims(st.mps) == mpsm.bond_dims(full)


def test_displaced_oscillator_stays_a_product():
    """No inter-state coupling: the exact state is a product, which is inside
    the D = 1 manifold, so 1TDVP at D = 1 follows the closed form."""
    om, ka = np.array([0.12, 0.2]), np.array([0.09, -0.14])
    model = synth.single_mode_model(om, ka, nbasis=30, E=(0.3, -0.2), state=0)
    psi0 = mpsm.product_state(ham.site_dims(model), model["occ"])
    st = tdvp.TDVP1(psi0, mpom.build_mpo(model))
    for k in range(1, 9):
        st.step(0.5)
        ref = exact.displaced_autocorrelation(0.5 * k, 0.3, om, ka)
        assert abs(obs.overlap(psi0, st.mps) - ref) < 1e-12
    assert max(mpsm.bond_dims(st.mps)) == 1


def test_rabi_oscillation_at_unit_bonds():
    model = synth.rabi_model(E0=0.0, E1=0.4, V01=0.05)
    st = tdvp.TDVP1(mpsm.product_state(ham.site_dims(model), model["occ"]), mpom.build_mpo(model))
    for k in range(1, 11):
        st.step(0.5)
        p = obs.populations(model, st.mps)
        assert abs(p[0] - exact.rabi_population(0.5 * k, 0.0, 0.4, 0.05)) < 1e-12


def test_norm_and_energy_conserved_at_fixed_bonds():
    """The paper's stated property of 1TDVP: no truncation, so the norm and
    the energy are conserved, here on bonds well below full rank."""
    model = synth.config1_model(2)
    mps, W = _grown(model, 3, 6)
    bonds = mpsm.bond_dims(mps)
    assert max(bonds) == 6 and bonds != mpsm.full_rank_caps(ham.site_dims(model))
    e0, n0 = obs.energy(mps, W), obs.norm2(mps)
    st = tdvp.TDVP1(mps, W)
    for _ in range(8):
        st.step(model["dt_fs"])
    assert abs(obs.norm2(st.mps) - n0) < 1e-12
    assert abs(obs.energy(st.mps, W) - e0) < 1e-11
    assert mpsm.bond_dims(st.mps) == bonds
    for a in st.mps[1:]:
        assert mpsm.right_orth_error(a) < 1e-12


def test_symmetric_step_is_time_reversible():
    """A forward step followed by the step with -dt returns the state: the
    right-to-left half-sweep is the inverse of the left-to-right one run
    backwards, at any bond dimension since nothing is truncated."""
    model = synth.config1_model(5)
    model["nbasis"] = np.array([4, 4, 4, 4])
    mps, W = _grown(model, 2, 5)
    v0 = mpsm.to_dense(mps)
    st = tdvp.TDVP1(mps, W)
    st.step(0.8)
    assert np.linalg.norm(mpsm.to_dense(st.mps) - v0) > 1e-3  # it moved
    st.step(-0.8)
    assert np.linalg.norm(mpsm.to_dense(st.mps) - v0) < 1e-10


def test_projection_error_shrinks_with_bond_dimension():
    """Below full rank 1TDVP carries a projection error; a larger frozen bond
    dimension gives a result closer to exact propagation."""
    model = _small_config1(1)
    psi0 = exact.product_vector(model)
    errs = []
    for D in (1, 2, 3, 4):
        mps, W = _grown(model, 2, D, dt=1.0)
        t0 = 2.0
        assert max(mpsm.bond_dims(mps)) == D
        st = tdvp.TDVP1(mps, W)
        for _ in range(4):
            st.step(0.5)
        ref = exact.evolve(model, psi0, [t0 + 2.0])[0]
        errs.append(np.linalg.norm(mpsm.to_dense(st.mps) - ref))
    assert errs[0] > errs[1] > errs[2] > errs[3]
