"""Whole-run pins of the oracle DMRG (CPU only)."""
import numpy as np
import pytest

from oracle import dmrg as OD
from oracle import models as M
from oracle import superblock as OS
from workloads import init_vector

from test_oracle_models import load_paper_energies


def _init(D, step):
    return init_vector(D, step)


def test_paper_test_run(golden_dir):
    """Hubbard U=1, m=64, infinite phase: the four printed energies."""
    log = OD.run(M.hubbard_model(1.0), 10, 64, 0, _init)
    got = {r["n"]: r["energy"] for r in log}
    for n, e in load_paper_energies(golden_dir):
        assert abs(got[n] - e) <= 5e-6, (n, got[n], e)
    # blocks of <= 3 sites are never truncated at m=64: exact up to n=8
    for n in (4, 6, 8):
        assert abs(got[n] - M.hubbard_ed(n, M.chain_bonds(n), 1.0)[0]) < 1e-9


def test_heisenberg_L16_m32_two_sweeps():
    log = OD.run(M.heisenberg_model(M.chain_bonds), 16, 32, 2, _init)
    e = log[-1]["energy"]
    ed = M.heisenberg_ed(16, M.chain_bonds(16))[0]
    assert e >= ed - 1e-10                 # variational
    assert (e - ed) / 16 < 1e-8
    assert log[-1]["phase"] == "finite" and log[-1]["p"] == 8


def test_hubbard_u4_exact_when_untruncated():
    log = OD.run(M.hubbard_model(4.0), 8, 64, 1, _init)
    ed = M.hubbard_ed(8, M.chain_bonds(8), 4.0)[0]
    assert abs(log[-1]["energy"] - ed) < 1e-9


def test_free_fermion_chain():
    L = 8
    log = OD.run(M.hubbard_model(0.0), L, 64, 1, _init)
    k = np.arange(1, L // 2 + 1)
    assert abs(log[-1]["energy"] - 2 * np.sum(-2 * np.cos(k * np.pi / (L + 1)))) < 1e-9


def test_majumdar_ghosh_chain():
    L = 16
    model = M.heisenberg_model(lambda n: M.j1j2_bonds(n, 1.0, 0.5))
    log = OD.run(model, L, 8, 1, _init)
    for r in log:
        assert abs(r["energy"] + 3 * r["n"] / 8) < 1e-9


def test_ladder_matches_ed():
    W = 4
    model = M.heisenberg_model(lambda n: M.ladder_bonds(n // 2))
    log = OD.run(model, 2 * W, 64, 1, _init)
    assert abs(log[-1]["energy"] - M.heisenberg_ed(2 * W, M.ladder_bonds(W))[0]) < 1e-9


def test_superblock_description_matches_dense_product():
    """The exported block-sparse superblock applies the same H as the dense one."""
    seen = []
    OD.run(M.hubbard_model(4.0), 8, 24, 0, _init,
           on_superblock=lambda ph, n, p, sb: seen.append(sb))
    sb = seen[-1]
    OS.check_quantum_numbers(sb)
    _, D = OS.target_pairs(sb)
    x = init_vector(D, 0)
    assert np.allclose(OS.hpsi_blocks(sb, x), OS.hpsi_dense(sb, x), atol=1e-12)


@pytest.mark.parametrize("name,model,L,m", [
    ("heisenberg", M.heisenberg_model(M.chain_bonds), 8, 256),
    ("j1j2", M.heisenberg_model(lambda n: M.j1j2_bonds(n, 1.0, 0.3)), 8, 256),
    ("hubbard_u4", M.hubbard_model(4.0), 6, 4096),
])
def test_carried_state_is_next_ground_state_when_untruncated(name, model, L, m):
    """Untruncated, the wave-function transformation is an exact change of
    basis of the same L-site state (the paper's conclusions, after White):
    the carried vector is the next step's ground state, in both sweep
    directions and at the turns."""
    log = OD.run(model, L, m, 1, _init, tol=1e-12)
    fin = [r for r in log if r["phase"] == "finite"]
    assert all(r.get("eps0", 0.0) == 0.0 and r.get("eps1", 0.0) == 0.0 for r in log)
    moved = [r for r in fin if "carry_overlap" in r]
    assert len(moved) == len(fin)
    for r in moved:
        assert r["carry_overlap"] >= 1 - 1e-10, (name, r["p"], r["carry_overlap"])
        assert abs(r["carry_energy"] - r["energy"]) <= 1e-9 * abs(r["energy"])


def test_carried_state_truncated_is_variational_and_close():
    """Truncated, the carried vector lies in the next superblock's space, so
    its energy is at least the next ground-state energy (variational), and
    it stays close to that ground state; starting Lanczos from it saves
    iterations against a random start."""
    model = M.heisenberg_model(M.chain_bonds)
    cold = OD.run(model, 16, 16, 1, _init)
    warm = OD.run(model, 16, 16, 1, _init, wavefunction=True)
    fin = [r for r in warm if r["phase"] == "finite"]
    assert all("carry_overlap" in r for r in fin)
    for r in fin:
        assert r["carry_energy"] >= r["energy"] - 1e-9 * abs(r["energy"])
        assert r["carry_overlap"] > 0.99, (r["p"], r["carry_overlap"])
    assert abs(warm[-1]["energy"] - cold[-1]["energy"]) < 1e-8
    it_cold = sum(r["iters"] for r in cold if r["phase"] == "finite")
    it_warm = sum(r["iters"] for r in fin)
    assert it_warm < 0.7 * it_cold, (it_warm, it_cold)
