"""Pins of the oracle's models and exact diagonalisation (CPU only).

Each check compares against something the oracle does not compute itself:
operator algebra, closed forms, the paper's printed energies, or a second,
independent construction of the same Hamiltonian.
"""
import numpy as np
import pytest

from oracle import models as M


def load_paper_energies(golden_dir):
    rows = []
    with open(golden_dir + "/paper_test_run_energies.txt") as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                n, e = line.split()
                rows.append((int(n), float(e)))
    return rows


def test_spin_algebra():
    s = M.spin_half_site()
    comm = s["Sp"] @ s["Sm"] - s["Sm"] @ s["Sp"]
    assert np.allclose(comm, 2 * s["Sz"])
    assert np.allclose(s["Sz"] @ s["Sp"] - s["Sp"] @ s["Sz"], s["Sp"])
    S2 = s["Sz"] @ s["Sz"] + 0.5 * (s["Sp"] @ s["Sm"] + s["Sm"] @ s["Sp"])
    assert np.allclose(S2, 0.75 * np.eye(2))


def test_site_fermion_algebra():
    s = M.hubbard_site()
    c = [s["c_up"], s["c_dn"]]
    for a in range(2):
        for b in range(2):
            anti = c[a] @ c[b].T + c[b].T @ c[a]
            assert np.allclose(anti, np.eye(4) * (a == b))
            assert np.allclose(c[a] @ c[b] + c[b] @ c[a], 0)
    # |updown> = c^dag_up c^dag_down |e>
    e = np.array([1.0, 0, 0, 0])
    assert np.allclose(c[0].T @ (c[1].T @ e), [0, 0, 0, 1])


@pytest.mark.parametrize("L", [2, 3])
def test_fock_space_anticommutation(L):
    c = M.fock_annihilators(L)
    n = 4 ** L
    I = np.eye(n)
    ops = [c[i][s].toarray() for i in range(L) for s in range(2)]
    for a, A in enumerate(ops):
        for b, B in enumerate(ops):
            assert np.allclose(A @ B.T + B.T @ A, I * (a == b))
            assert np.allclose(A @ B + B @ A, 0)


@pytest.mark.parametrize("J", [1.0, 2.5])
def test_two_site_heisenberg_singlet(J):
    assert abs(M.heisenberg_ed(2, M.chain_bonds(2, J))[0] - (-0.75 * J)) < 1e-13


@pytest.mark.parametrize("U,t", [(0.0, 1.0), (1.0, 1.0), (4.0, 1.0), (8.0, 0.5)])
def test_two_site_hubbard_closed_form(U, t):
    e = M.hubbard_ed(2, M.chain_bonds(2, t), U)[0]
    assert abs(e - (U - np.sqrt(U * U + 16 * t * t)) / 2) < 1e-12


def test_four_site_heisenberg_closed_form():
    # open 4-site chain: E0 = -(3 + 2 sqrt 3) / 4
    assert abs(M.heisenberg_ed(4, M.chain_bonds(4))[0] + (3 + 2 * np.sqrt(3)) / 4) < 1e-12


@pytest.mark.parametrize("L,t", [(4, 1.0), (6, 1.0), (8, 0.7), (10, 1.0)])
def test_free_fermions(L, t):
    k = np.arange(1, L // 2 + 1)
    exact = 2 * np.sum(-2 * t * np.cos(k * np.pi / (L + 1)))
    assert abs(M.hubbard_ed(L, M.chain_bonds(L, t), 0.0)[0] - exact) < 1e-10


def test_paper_test_run_energies(golden_dir):
    for n, e in load_paper_energies(golden_dir):
        ed = M.hubbard_ed(n, M.chain_bonds(n), 1.0)[0]
        assert abs(ed - e) <= 5e-6, (n, ed, e)


@pytest.mark.parametrize("L", [8, 10, 12])
def test_majumdar_ghosh(L):
    w = M.heisenberg_ed(L, M.j1j2_bonds(L, 1.0, 0.5), k=2)
    assert abs(w[0] + 3 * L / 8) < 1e-10
    assert w[1] - w[0] > 0.1          # unique ground state


def test_decoupled_rungs():
    W = 4
    assert abs(M.heisenberg_ed(2 * W, M.ladder_bonds(W, 0.0, 1.0))[0] + 0.75 * W) < 1e-12


def test_large_u_hubbard_is_heisenberg():
    # half filling, U >> t: H_eff = J sum (S_i.S_j - 1/4), J = 4 t^2 / U
    L, U = 6, 200.0
    J = 4.0 / U
    eh = M.hubbard_ed(L, M.chain_bonds(L), U)[0]
    es = M.heisenberg_ed(L, M.chain_bonds(L, J))[0] - 0.25 * J * (L - 1)
    assert abs(eh - es) / abs(es) < 1e-3


@pytest.mark.parametrize("L", [2, 3, 4])
def test_kron_hamiltonian_matches_bitstrings(L):
    H = M.hubbard_fock_hamiltonian(L, M.chain_bonds(L), 2.0, V=0.3)
    nu, nd = M.hubbard_fock_numbers(L)
    for a in range(L + 1):
        for b in range(L + 1):
            idx = np.nonzero((nu == a) & (nd == b))[0]
            w1 = np.linalg.eigvalsh(H[idx][:, idx].toarray())
            w2 = np.linalg.eigvalsh(M.hubbard_sector_matrix(L, M.chain_bonds(L), 2.0, a, b,
                                                            V=0.3).toarray())
            assert np.allclose(w1, w2, atol=1e-11)
    # the Hamiltonian conserves (N_up, N_down)
    Hd = H.toarray()
    mism = (nu[:, None] != nu[None, :]) | (nd[:, None] != nd[None, :])
    assert np.all(Hd[mism] == 0)


def test_kron_heisenberg_matches_bitstrings():
    L = 6
    bonds = M.j1j2_bonds(L, 1.0, 0.3)
    H = M.heisenberg_kron_hamiltonian(L, bonds).toarray()
    n = M.spin_kron_nup(L)
    for k in range(L + 1):
        idx = np.nonzero(n == k)[0]
        w1 = np.linalg.eigvalsh(H[np.ix_(idx, idx)])
        w2 = np.linalg.eigvalsh(M.heisenberg_sector_matrix(L, bonds, k).toarray())
        assert np.allclose(w1, w2, atol=1e-11)
