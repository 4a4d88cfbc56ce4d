"""CPU check of the whole-run driver's orchestration, with the oracle standing
in for the library (test only): every product, ground state and truncation
is the oracle's, so the driver's own bookkeeping -- growth, basis change
plumbing, finite-sweep order, and the wave-function transformation between
steps -- is what is tested.
"""
import numpy as np
import pytest
import torch

from oracle import lanczos as OL
from oracle import models as M
from oracle import rho as OR
from oracle import superblock as OS
from workloads import init_vector


class FakeContext:
    def transform_blocks(self, blocks, O, W, out):
        Oh, Wh = O.numpy(), W.numpy()
        o = out.numpy()
        for b in blocks:
            r, c, kr, kc = b["rows"], b["cols"], b["kr"], b["kc"]
            old = b.get("o_ld", 0) or c
            oud = b.get("out_ld", 0) or kc
            Ob = np.lib.stride_tricks.as_strided(Oh[b["o_off"]:], (r, c), (old * 8, 8))
            Wr = Wh[b["wr_off"]:b["wr_off"] + r * kr].reshape(r, kr)
            Wc = Wh[b["wc_off"]:b["wc_off"] + c * kc].reshape(c, kc)
            res = OR.transform_block(Ob, Wr, Wc)
            for i in range(kr):
                o[b["out_off"] + i * oud:b["out_off"] + i * oud + kc] = res[i]
        return out


STARTS = []


class FakeSuperblock:
    def __init__(self, desc, prec="fp64", ctx=None):
        self.desc = desc
        pairs, self.D = OS.target_pairs(desc)
        self.s_sec = np.array([p[0] for p in pairs])
        self.e_sec = np.array([p[1] for p in pairs])
        self.offsets = np.array([p[2] for p in pairs])
        self._dims = (np.asarray(desc["S"]["dim"]), np.asarray(desc["E"]["dim"]))

    def lanczos(self, psi0, max_iter=300, tol=1e-10):
        v0 = psi0.numpy().copy()
        E, psi, it, res = OL.lanczos_ground(lambda v: OS.hpsi_blocks(self.desc, v), v0,
                                            max_iter=max_iter, tol=1e-12)
        STARTS.append(abs(np.dot(v0, psi)) / np.linalg.norm(v0))
        return dict(energy=E, psi=torch.tensor(psi), iters=it, resid=res)

    def rho_truncate(self, psi, side, m, no_split=False):
        return OR.truncate(self.desc, psi.numpy(), side, m, no_split=no_split)

    def close(self):
        pass


@pytest.fixture
def fake(monkeypatch):
    from paper_0902_3185_amd import driver as DR
    from paper_0902_3185_amd import superblock as SBM
    monkeypatch.setattr(DR, "DEVICE", "cpu")
    monkeypatch.setattr(SBM, "Superblock", FakeSuperblock)
    STARTS.clear()
    return DR


def _init(D, step):
    return init_vector(D, step)


def test_untruncated_run_is_exact_and_transformed_start_is_the_ground_state(fake):
    DR = fake
    L = 8
    log = DR.run(DR.hubbard(2.0), L, 1000, 1, _init, ctx=FakeContext(), tol=1e-12)
    ed = M.hubbard_ed(L, M.chain_bonds(L), 2.0)[0]
    for r in log:
        if r["phase"] == "finite":
            assert abs(r["energy"] - ed) < 1e-10
    n_inf = sum(1 for r in log if r["phase"] == "infinite")
    # without truncation every carried start vector is the exact ground state
    assert len(STARTS) == len(log)
    assert min(STARTS[n_inf:]) > 1 - 1e-10


def test_truncated_run_matches_oracle_and_starts_are_good(fake):
    DR = fake
    L = 12
    log = DR.run(DR.heisenberg(DR.chain(1.0)), L, 12, 1, _init, ctx=FakeContext(), tol=1e-12)
    from oracle import dmrg as OD
    ref = OD.run(M.heisenberg_model(M.chain_bonds), L, 12, 1, _init, tol=1e-11)
    for a, b in zip(log, ref):
        assert abs(a["energy"] - b["energy"]) < 1e-9 * L
    n_inf = sum(1 for r in log if r["phase"] == "infinite")
    assert min(STARTS[n_inf:]) > 0.99


def test_transformation_off_gives_same_energies(fake):
    DR = fake
    L = 10
    a = DR.run(DR.heisenberg(DR.j1j2(1.0, 0.3)), L, 10, 1, _init, ctx=FakeContext(), tol=1e-12)
    b = DR.run(DR.heisenberg(DR.j1j2(1.0, 0.3)), L, 10, 1, _init, ctx=FakeContext(), tol=1e-12,
               wavefunction=False)
    for x, y in zip(a, b):
        assert abs(x["energy"] - y["energy"]) < 1e-9 * L


@pytest.mark.parametrize("bonds", ["chain", "j1j2", "ladder"])
def test_reflection_in_infinite_phase(fake, bonds):
    """Environment = mirrored system block: same energies, half the truncations."""
    DR = fake
    L = 12
    bf = {"chain": DR.chain(1.0), "j1j2": DR.j1j2(1.0, 0.4), "ladder": DR.ladder(1.0, 0.7)}[bonds]
    a = DR.run(DR.heisenberg(bf), L, 16, 1, _init, ctx=FakeContext(), tol=1e-12, reflect=True)
    b = DR.run(DR.heisenberg(bf), L, 16, 1, _init, ctx=FakeContext(), tol=1e-12, reflect=False)
    for x, y in zip(a, b):
        assert abs(x["energy"] - y["energy"]) < 1e-9 * L, (x, y)
    assert all("eps1" not in r for r in a if r["phase"] == "infinite")
    n_inf = sum(1 for r in a if r["phase"] == "infinite")
    assert min(STARTS[n_inf:len(a)]) > 0.99   # run a's finite steps only


@pytest.mark.parametrize("U", [4.0, 0.0])
def test_reflection_for_fermions(fake, U):
    """Hubbard chain (spinful fermions): the mirrored system block, with the
    sign of reversing each configuration's operator order in its basis,
    serves as the environment with the system block's own matrices -- the
    energies agree with the explicit environment's, and the carried start
    vectors, which go through the mirrored blocks' cut records (sign
    (-1)^(N_a n_x) per row), stay close to the ground states."""
    DR = fake
    assert DR.mirror_symmetric(DR.hubbard(U), 8)
    assert DR.mirror_symmetric(DR.heisenberg(DR.ladder()), 8)
    L = 10
    a = DR.run(DR.hubbard(U), L, 24, 1, _init, ctx=FakeContext(), tol=1e-12, reflect=True)
    starts = list(STARTS)
    b = DR.run(DR.hubbard(U), L, 24, 1, _init, ctx=FakeContext(), tol=1e-12, reflect=False)
    assert len(a) == len(b)
    for x, y in zip(a, b):
        assert abs(x["energy"] - y["energy"]) < 1e-12 * L, (x, y)
    assert all("eps1" not in r for r in a if r["phase"] == "infinite")
    n_inf = sum(1 for r in a if r["phase"] == "infinite")
    assert min(starts[n_inf:]) > 0.999


def test_checkpoint_and_resume(fake, tmp_path):
    """A run stopped after nine steps (inside the finite sweep) with
    checkpoints, then resumed from them: the saved records come back as they
    were, the remaining steps give the uninterrupted run's energies, and the
    resumed steps after the first start from carried vectors close to their
    ground states (the blocks' cut records were saved with them)."""
    DR = fake
    L = 12
    model = DR.heisenberg(DR.chain(1.0))
    full = DR.run(model, L, 12, 1, _init, ctx=FakeContext(), tol=1e-12)
    pre = str(tmp_path / "ck")
    part = DR.run(model, L, 12, 1, _init, ctx=FakeContext(), tol=1e-12, checkpoint=pre, stop_after=9)
    assert len(part) == 9
    STARTS.clear()
    rest = DR.run(model, L, 12, 1, _init, ctx=FakeContext(), tol=1e-12, resume=pre)
    assert len(rest) == len(full)
    for a, b in zip(rest[:9], part):
        assert a == b
    for a, b in zip(rest, full):
        assert (a["phase"], a["n"], a["p"]) == (b["phase"], b["n"], b["p"])
        assert abs(a["energy"] - b["energy"]) < 1e-10 * L
    assert len(STARTS) == len(full) - 9
    assert min(STARTS[1:]) > 0.99
