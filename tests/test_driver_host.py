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


def _same_desc(a, b):
    for side in ("S", "E"):
        assert np.array_equal(a[side]["q"], b[side]["q"]) and np.array_equal(a[side]["dim"], b[side]["dim"])
    assert a["q_target"] == b["q_target"] and len(a["terms"]) == len(b["terms"])
    for ta, tb in zip(a["terms"], b["terms"]):
        assert ta["c"] == tb["c"] and ta.get("group", 0) == tb.get("group", 0)
        for side in ("A", "B"):
            if ta[side] is None:
                assert tb[side] is None
                continue
            assert ta[side]["delta"] == tb[side]["delta"]
            assert len(ta[side]["blocks"]) == len(tb[side]["blocks"])
            for (r, c, x), (r2, c2, y) in zip(ta[side]["blocks"], tb[side]["blocks"]):
                assert (r, c) == (r2, c2) and np.array_equal(np.asarray(x, dtype=np.float64), y)


def test_superblock_fixture_round_trip(tmp_path):
    """checkpoint.save_superblock / load_superblock keep every sector, term
    and block bit for bit (and the vector beside them), so a loaded fixture
    describes the same operator."""
    from paper_0902_3185_amd import checkpoint as CK
    from workloads import seeded_vector, workload_superblock
    model = DR.hubbard(4.0)
    S, E, Q, bonds = _grown(model, 6)
    nu, nd = model.target(6)
    cases = [DR.superblock(S, E, model, Q, 6, bonds, nu + Q * nd),
             workload_superblock("heisenberg_L16_m32", seed=2)]
    for k, desc in enumerate(cases):
        _, D = OS.target_pairs(desc)
        psi = seeded_vector(D, 11)
        path = tmp_path / f"sb{k}.npz"
        CK.save_superblock(path, desc, psi)
        back, psi2 = CK.load_superblock(path)
        _same_desc(desc, back)
        assert np.array_equal(psi, psi2)
        assert np.array_equal(OS.hpsi_blocks(desc, psi), OS.hpsi_blocks(back, psi))
    CK.save_superblock(tmp_path / "nopsi.npz", cases[0])
    assert CK.load_superblock(tmp_path / "nopsi.npz")[1] is None


def test_block_stack_round_trip(tmp_path):
    """checkpoint.save_blocks / load_blocks: labels, sectors, Hamiltonian
    and operator blocks bit for bit, the run state as written, and a
    truncated block's cut record (its product rebuilt from the two bases,
    the kept vectors per sector)."""
    from paper_0902_3185_amd import checkpoint as CK
    model = DR.hubbard(4.0)
    Q = 9
    bonds = model.bonds(8)
    S1 = DR.site_block(model, 0, Q)
    S2 = DR.grow_right(S1, model, Q, bonds, 1)
    S3 = DR.grow_right(S2, model, Q, bonds, 1)
    rng = np.random.default_rng(4)
    kept = [(s, rng.standard_normal((int(S3.product.basis.dim[s]), 1)))
            for s in range(0, len(S3.product.basis.q), 2)]
    S3.origin = (S3.product, kept)
    state = dict(done=3, log=[dict(energy=-1.5, iters=np.int64(7))])
    path = tmp_path / "run.blocks.npz"
    CK.save_blocks(path, {"left": {1: S1, 2: S2, 3: S3}, "right": {1: S1}}, state)
    stacks, st = CK.load_blocks(path)
    assert st == dict(done=3, log=[dict(energy=-1.5, iters=7)])
    assert sorted(stacks["left"]) == [1, 2, 3] and sorted(stacks["right"]) == [1]
    for pos, blk in ((1, S1), (2, S2), (3, S3)):
        got = stacks["left"][pos]
        assert got.labels == blk.labels
        assert np.array_equal(got.basis.q, blk.basis.q) and np.array_equal(got.basis.dim, blk.basis.dim)
        assert sorted(got.H) == sorted(blk.H)
        for g in blk.H:
            assert sorted(got.H[g]) == sorted(blk.H[g])
            for key, b in blk.H[g].items():
                assert np.array_equal(got.H[g][key], b)
        assert sorted(got.ops) == sorted(blk.ops)
        for key, op in blk.ops.items():
            assert got.ops[key].delta == op.delta and sorted(got.ops[key].blocks) == sorted(op.blocks)
            for bk, b in op.blocks.items():
                assert np.array_equal(got.ops[key].blocks[bk], b)
    assert stacks["left"][2].origin is None
    P, kept2 = stacks["left"][3].origin
    assert P.runs == S3.product.runs and np.array_equal(P.basis.dim, S3.product.basis.dim)
    assert [s for s, _ in kept2] == [s for s, _ in kept]
    assert all(np.array_equal(a, b) for (_, a), (_, b) in zip(kept, kept2))


def test_checkpoint_refuses_other_formats(tmp_path):
    import json
    from paper_0902_3185_amd import checkpoint as CK
    path = tmp_path / "bad.npz"
    np.savez(path, header=np.array(json.dumps(dict(format=99, kind="blocks"))))
    with pytest.raises(ValueError):
        CK.load_blocks(path)
    np.savez(path, header=np.array(json.dumps(dict(format=CK.FORMAT, kind="blocks", index={}, state=None))))
    with pytest.raises(ValueError):
        CK.load_superblock(path)
