"""The stored physical superblock (Hubbard chain L=64, U=4, m=512, the centre
superblock of the oracle's infinite-phase run, written by
oracle/write_physical_fixture.py): both readers agree, its quantum numbers
are consistent, and its ground energy is the one the oracle's run recorded
for that step."""
import os

import numpy as np
import pytest

from oracle import lanczos as OL
from oracle import superblock as OS
from workloads import seeded_vector
from workloads.superblocks import DATA, FIXTURES, fixture_superblock

NAME = "hubbard_L64_U4_m512_physical"
pytestmark = pytest.mark.skipif(not os.path.exists(os.path.join(DATA, FIXTURES[NAME])),
                                reason="fixture file not present")


def test_readers_agree():
    from paper_0902_3185_amd import checkpoint as CK
    a = fixture_superblock(NAME)
    b, psi = CK.load_superblock(os.path.join(DATA, FIXTURES[NAME]))
    assert psi is None
    for side in ("S", "E"):
        assert np.array_equal(a[side]["q"], b[side]["q"]) and np.array_equal(a[side]["dim"], b[side]["dim"])
    assert a["q_target"] == b["q_target"] and len(a["terms"]) == len(b["terms"])
    for ta, tb in zip(a["terms"], b["terms"]):
        assert (ta["c"], ta["group"]) == (tb["c"], tb["group"])
        for side in ("A", "B"):
            assert (ta[side] is None) == (tb[side] is None)
            if ta[side] is not None:
                assert ta[side]["delta"] == tb[side]["delta"]
                for (r, c, x), (r2, c2, y) in zip(ta[side]["blocks"], tb[side]["blocks"]):
                    assert (r, c) == (r2, c2) and np.array_equal(x, y)


def test_physical_superblock_ground_energy():
    desc = fixture_superblock(NAME)
    meta = desc["meta"]
    assert (meta["model"], meta["L"], meta["U"], meta["m"]) == ("hubbard", 64, 4.0, 512)
    OS.check_quantum_numbers(desc)
    _, D = OS.target_pairs(desc)
    E, psi, it, res = OL.lanczos_ground(lambda v: OS.hpsi_blocks(desc, v), seeded_vector(D, 0),
                                        max_iter=600, tol=1e-9)
    assert res <= 1e-9
    # the energy the run recorded for its last step (same superblock, same
    # solver, another start vector)
    assert abs(E - meta["energies"][-1]) <= 1e-8 * 64, (E, meta["energies"][-1])
    # half-filled Hubbard chain at U = 4: the energy per site of the open
    # 64-site chain lies a boundary correction above the infinite chain's
    # -0.5737 (Lieb-Wu)
    assert -0.5737 < E / 64 < -0.55, E / 64
