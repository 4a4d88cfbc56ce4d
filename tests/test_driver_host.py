"""CPU checks of the whole-run driver's host block algebra (no device calls).

An untruncated superblock built by the driver (block-sparse growth, bond
terms with fermion parity) must have the exact ground energy of the chain;
the oracle's explicit Kronecker matrix is used only as the checker.
"""
import numpy as np
import pytest

from oracle import models as M
from oracle import superblock as OS
from paper_0902_3185_amd import driver as DR


def _grown(model, L):
    Q = L + 1
    bonds = model.bonds(L)
    keep = max(j - i for (i, j, _v, _g) in bonds)
    S = DR.site_block(model, 0, Q)
    E = DR.site_block(model, 0, Q)
    for _ in range(L // 2 - 1):
        S = DR.grow_right(S, model, Q, bonds, keep)
        E = DR.grow_left(E, model, Q, L, bonds, keep)
    return S, E, Q, bonds


@pytest.mark.parametrize("L,U", [(4, 1.0), (6, 4.0), (6, 0.0)])
def test_hubbard_superblock_is_exact(L, U):
    model = DR.hubbard(U)
    S, E, Q, bonds = _grown(model, L)
    nu, nd = model.target(L)
    desc = DR.superblock(S, E, model, Q, L, bonds, nu + Q * nd)
    OS.check_quantum_numbers(desc)
    e0 = np.linalg.eigvalsh(OS.kron_matrix(desc))[0]
    assert abs(e0 - M.hubbard_ed(L, M.chain_bonds(L), U)[0]) < 1e-11


@pytest.mark.parametrize("name,L", [("chain", 8), ("j1j2", 8), ("ladder", 8)])
def test_spin_superblock_is_exact(name, L):
    bonds_fn = {"chain": DR.chain(1.0), "j1j2": DR.j1j2(1.0, 0.35), "ladder": DR.ladder(0.8, 1.0)}[name]
    model = DR.heisenberg(bonds_fn)
    S, E, Q, bonds = _grown(model, L)
    desc = DR.superblock(S, E, model, Q, L, bonds, L // 2)
    OS.check_quantum_numbers(desc)
    e0 = np.linalg.eigvalsh(OS.kron_matrix(desc))[0]
    ref = {"chain": M.chain_bonds(L), "j1j2": M.j1j2_bonds(L, 1.0, 0.35),
           "ladder": M.ladder_bonds(L // 2, 0.8, 1.0)}[name]
    assert abs(e0 - M.heisenberg_ed(L, ref)[0]) < 1e-11


def test_block_hamiltonian_is_symmetric_and_q_diagonal():
    model = DR.hubbard(2.0)
    S, E, Q, bonds = _grown(model, 6)
    for g, blocks in S.H.items():
        for (r, c), b in blocks.items():
            assert r == c
            assert np.allclose(b, b.T)
