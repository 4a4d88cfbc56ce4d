"""Pins of the oracle's local density of states (Eq. (5))."""
import numpy as np

from oracle import ldos as OLD
from oracle import models as M


def test_free_fermion_removal_spectrum_closed_form():
    """U = 0: removing an up electron from site i leaves a hole in an occupied
    orbital k with energy eps_k = -2t cos(k pi/(L+1)) and weight |phi_k(i)|^2,
    phi_k(i) = sqrt(2/(L+1)) sin(k pi (i+1)/(L+1))."""
    L, i, eta = 8, 2, 0.07
    omega = np.linspace(-3, 3, 61)
    N, e0, w, poles = OLD.hubbard_ldos_lehmann(L, M.chain_bonds(L), 0.0, i, 0, omega, eta)
    k = np.arange(1, L // 2 + 1)
    eps = -2 * np.cos(k * np.pi / (L + 1))
    wk = 2 / (L + 1) * np.sin(k * np.pi * (i + 1) / (L + 1)) ** 2
    ref = np.array([2 * np.pi * np.sum(wk * OLD.lorentzian(om - eps, eta)) for om in omega])
    assert np.max(np.abs(N - ref)) < 1e-10 * np.max(ref)


def test_sum_rule_half_filling():
    """sum_n |<n|c_i|psi>|^2 = <n_i,up> = 1/2 at half filling (particle-hole symmetry)."""
    L = 6
    for U in (1.0, 4.0):
        for site in range(L):
            _, _, w, _ = OLD.hubbard_ldos_lehmann(L, M.chain_bonds(L), U, site, 0, [0.0], 0.1)
            assert abs(np.sum(w) - 0.5) < 1e-12


def test_continued_fraction_equals_lehmann():
    L, U, site, eta = 6, 1.0, 2, 0.1
    omega = np.linspace(-4, 4, 81)
    N, e0, w, poles = OLD.hubbard_ldos_lehmann(L, M.chain_bonds(L), U, site, 1, omega, eta)
    n = L // 2
    H = M.hubbard_sector_matrix(L, M.chain_bonds(L), U, n, n).toarray()
    vals, vecs = np.linalg.eigh(H)
    H2 = M.hubbard_sector_matrix(L, M.chain_bonds(L), U, n, n - 1).toarray()
    phi = OLD.annihilator_bits(L, n, n, site, 1) @ vecs[:, 0]
    a, b, nrm = OLD.lanczos_coefficients(lambda v: H2 @ v, phi, H2.shape[0])
    cf = OLD.ldos_continued_fraction(a, b, nrm ** 2, vals[0], omega, eta)
    assert np.max(np.abs(cf - N)) < 1e-9 * np.max(N)
