"""Pins of the oracle's damped autocorrelation spectrum (the spectra of the
paper's Section 3.1): the closed-form geometric sum of a single level, the
continuous Lorentzian within the trapezoid rule's error bound, the exact
sum rule over one period of the sampled transform, and the Franck-Condon
progression of displaced oscillators."""
import numpy as np

from oracle import HBAR, exact
from oracle import observables as obs


def test_single_level_is_a_geometric_sum():
    """C(t) = exp(-i E0 t / hbar): the trapezoid sum of exp(a t_k) is
    dt [(1 - r^N) / (1 - r) - (1 + r^(N-1)) / 2] with r = exp(a dt)."""
    E0, dt, N, tau = 0.35, 0.5, 400, 30.0
    t = dt * np.arange(N)
    C = np.exp(-1j * E0 * t / HBAR)
    E = np.linspace(0.0, 0.8, 81)
    got = obs.absorption_spectrum(C, dt, E, tau)
    a = 1j * (E - E0) / HBAR - 1.0 / tau
    r = np.exp(a * dt)
    ref = (dt * ((1 - r ** N) / (1 - r) - 0.5 * (1 + r ** (N - 1)))).real / (np.pi * HBAR)
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


def test_single_level_lorentzian_within_trapezoid_bound():
    E0, dt, N, tau = 0.35, 0.05, 8001, 30.0
    T = dt * (N - 1)
    t = dt * np.arange(N)
    C = np.exp(-1j * E0 * t / HBAR)
    E = np.linspace(0.2, 0.5, 31)
    got = obs.absorption_spectrum(C, dt, E, tau)
    a = 1j * (E - E0) / HBAR - 1.0 / tau
    ref = ((np.exp(a * T) - 1) / a).real / (np.pi * HBAR)
    bound = T * dt ** 2 * np.abs(a) ** 2 / 12 / (np.pi * HBAR)  # |f''| <= |a|^2 on [0, T]
    assert np.all(np.abs(got - ref) <= bound + 1e-14)
    # and the peak is the Lorentzian height tau / (pi hbar) up to exp(-T / tau)
    peak = obs.absorption_spectrum(C, dt, [E0], tau)[0]
    assert abs(peak - tau / (np.pi * HBAR)) < 2e-4 * tau / (np.pi * HBAR)


def test_sum_rule_over_one_period():
    """sum_m sigma(E_m) dE over M > N - 1 equally spaced points of one
    period 2 pi hbar / dt equals Re C(0) exactly (only the t = 0 term
    survives, with trapezoid weight dt / 2)."""
    rng = np.random.default_rng(0)
    N, dt = 64, 0.5
    C = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    M = 200
    period = 2 * np.pi * HBAR / dt
    E = -1.3 + period * np.arange(M) / M
    s = obs.absorption_spectrum(C, dt, E, 1e300)  # no damping
    assert abs(s.sum() * period / M - C[0].real) < 1e-12 * np.abs(C).max() * N


def test_displaced_oscillator_franck_condon_progression():
    """One displaced mode from the vacuum: C(t) = exp(-i E t/hbar) exp(-i w t/2hbar
    + i S w t/hbar - S (1 - exp(-i w t/hbar))) = sum_n e^{-S} S^n / n! exp(-i E_n t/hbar)
    with E_n = E + w/2 - S w + n w, so the spectrum is the Poisson-weighted sum
    of single-level spectra."""
    from math import factorial
    E, w, k = 0.3, 0.12, 0.09
    S = k * k / (2 * w * w)
    dt, N, tau = 0.25, 2000, 30.0
    t = dt * np.arange(N)
    C = exact.displaced_autocorrelation(t, E, [w], [k])
    grid = np.linspace(0.1, 0.9, 161)
    got = obs.absorption_spectrum(C, dt, grid, tau)
    ref = np.zeros_like(grid)
    for n in range(40):
        En = E + w / 2 - S * w + n * w
        ref += np.exp(-S) * S ** n / factorial(n) * obs.absorption_spectrum(np.exp(-1j * En * t / HBAR), dt, grid, tau)
    assert np.abs(got - ref).max() < 1e-10 * np.abs(ref).max()
