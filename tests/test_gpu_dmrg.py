"""Whole DMRG runs through the library (GPU) against the oracle, exact
diagonalisation and the paper's printed energies."""
import numpy as np
import pytest

from oracle import dmrg as OD
from oracle import models as M
from workloads import init_vector

from test_oracle_models import load_paper_energies

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_0902_3185_amd.superblock import Context
    return Context(0)


def _init(D, step):
    return init_vector(D, step)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_paper_test_run(ctx, golden_dir, prec):
    """Hubbard U=1, m=64: the Test Run section's energies at n = 4..10."""
    from paper_0902_3185_amd import driver as DR
    log = DR.run(DR.hubbard(1.0), 10, 64, 0, _init, ctx=ctx, prec=prec, tol=1e-9)
    got = {r["n"]: r["energy"] for r in log}
    for n, e in load_paper_energies(golden_dir):
        assert abs(got[n] - e) <= 5e-6, (n, got[n], e)
    for n in (4, 6, 8):
        assert abs(got[n] - M.hubbard_ed(n, M.chain_bonds(n), 1.0)[0]) <= 1e-9 * n


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_heisenberg_L16_m32_matches_oracle_run(ctx, prec):
    from paper_0902_3185_amd import driver as DR
    L = 16
    log = DR.run(DR.heisenberg(DR.chain(1.0)), L, 32, 2, _init, ctx=ctx, prec=prec, tol=1e-9)
    ref = OD.run(M.heisenberg_model(M.chain_bonds), L, 32, 2, _init, tol=1e-10)
    assert len(log) == len(ref)
    for a, b in zip(log, ref):
        assert abs(a["energy"] - b["energy"]) <= 1e-9 * L, (a, b)
        assert abs(a.get("eps0", 0.0) - b.get("eps0", 0.0)) <= 1e-9
    ed = M.heisenberg_ed(L, M.chain_bonds(L))[0]
    assert log[-1]["energy"] >= ed - 1e-10 and (log[-1]["energy"] - ed) / L < 1e-8


def test_majumdar_ghosh(ctx):
    from paper_0902_3185_amd import driver as DR
    log = DR.run(DR.heisenberg(DR.j1j2(1.0, 0.5)), 20, 8, 1, _init, ctx=ctx, prec="fp32", tol=1e-9)
    for r in log:
        assert abs(r["energy"] + 3 * r["n"] / 8) <= 1e-9 * r["n"]


def test_hubbard_u4_and_ladder_exact(ctx):
    from paper_0902_3185_amd import driver as DR
    log = DR.run(DR.hubbard(4.0), 8, 64, 1, _init, ctx=ctx, prec="fp64", tol=1e-10)
    assert abs(log[-1]["energy"] - M.hubbard_ed(8, M.chain_bonds(8), 4.0)[0]) < 1e-9
    log = DR.run(DR.heisenberg(DR.ladder(1.0, 1.0)), 8, 64, 1, _init, ctx=ctx, prec="fp32", tol=1e-9)
    assert abs(log[-1]["energy"] - M.heisenberg_ed(8, M.ladder_bonds(4))[0]) < 1e-9


def test_wavefunction_transformation_saves_products(ctx):
    """Carrying psi between finite-sweep steps (on the GPU) leaves the energies
    unchanged and cuts the number of products."""
    from paper_0902_3185_amd import driver as DR
    L = 16
    a = DR.run(DR.heisenberg(DR.chain(1.0)), L, 32, 1, _init, ctx=ctx, prec="fp32", tol=1e-9)
    b = DR.run(DR.heisenberg(DR.chain(1.0)), L, 32, 1, _init, ctx=ctx, prec="fp32", tol=1e-9,
               wavefunction=False)
    for x, y in zip(a, b):
        assert abs(x["energy"] - y["energy"]) <= 1e-9 * L
    fa = sum(r["iters"] for r in a if r["phase"] == "finite")
    fb = sum(r["iters"] for r in b if r["phase"] == "finite")
    assert fa < 0.6 * fb, (fa, fb)


def test_reflection_on_gpu(ctx):
    from paper_0902_3185_amd import driver as DR
    L = 16
    a = DR.run(DR.heisenberg(DR.chain(1.0)), L, 32, 1, _init, ctx=ctx, prec="fp32", tol=1e-9,
               reflect=True)
    ref = OD.run(M.heisenberg_model(M.chain_bonds), L, 32, 1, _init, tol=1e-10)
    assert abs(a[-1]["energy"] - ref[-1]["energy"]) <= 1e-9 * L


def test_fermion_reflection_on_gpu(ctx):
    """Hubbard U=4 (spinful fermions) with the mirrored environment in the
    infinite phase: every step's energy is the oracle run's (explicit
    environment), and the finite sweep that follows, which carries its
    start vectors through the mirrored blocks, ends at the oracle's too."""
    from paper_0902_3185_amd import driver as DR
    L = 12
    a = DR.run(DR.hubbard(4.0), L, 64, 1, _init, ctx=ctx, prec="fp64", tol=1e-10, reflect=True)
    ref = OD.run(M.hubbard_model(4.0), L, 64, 1, _init, tol=1e-10)
    assert len(a) == len(ref)
    assert all("eps1" not in r for r in a if r["phase"] == "infinite")
    for x, y in zip(a, ref):
        assert abs(x["energy"] - y["energy"]) <= 1e-9 * L, (x, y)


@pytest.mark.parametrize("U,spin", [(1.0, 0), (4.0, 1)])
def test_ldos_matches_exact_diagonalisation(ctx, U, spin):
    """Eq. (5) on the centre superblock of an untruncated 8-site Hubbard run:
    continued fraction through the library vs the ED Lehmann sum."""
    from oracle import ldos as OLD
    from paper_0902_3185_amd import driver as DR
    L = 8
    keep = {}
    DR.run(DR.hubbard(U), L, 256, 1, _init, ctx=ctx, prec="fp64", tol=1e-11,
           on_solve=lambda Sp, Ep, n, desc, r: keep.update(Sp=Sp, Ep=Ep, n=n, desc=desc, r=r))
    Sp, Ep, desc, r = keep["Sp"], keep["Ep"], keep["desc"], keep["r"]
    site = max(Sp.labels)
    omega = np.linspace(-4, 4, 81)
    eta = 0.1
    N = DR.ldos(ctx, Sp, Ep, DR.hubbard(U), L, desc["q_target"], r["psi"], site, spin, omega,
                eta, nsteps=800)
    ref, _, w, _ = OLD.hubbard_ldos_lehmann(L, M.chain_bonds(L), U, site, spin, omega, eta)
    assert np.max(np.abs(N - ref)) <= 1e-9 * np.max(ref)


def test_ladder_decoupled_rungs_stated_size(ctx):
    """Two-leg ladder 2x32 (L = 64, snake order) with J_leg = 0, m = 1024:
    the rungs decouple, the ground state is the product of rung singlets and
    every infinite-phase step must give E = -3n/8 (E = -24 at n = 64)."""
    from paper_0902_3185_amd import driver as DR
    log = DR.run(DR.heisenberg(DR.ladder(0.0, 1.0)), 64, 1024, 0, _init, ctx=ctx, prec="fp32",
                 tol=1e-9)
    assert log[-1]["n"] == 64
    for r in log:
        assert abs(r["energy"] + 3 * r["n"] / 8) <= 1e-9 * r["n"], r


def test_free_fermion_hubbard_stated_size(ctx):
    """Hubbard chain L = 64 at U = 0, m = 512 (infinite phase, FP32 products
    with FP64 cycles): the energy is variational and within 1e-6 per site
    of the free-fermion closed form 2 sum_k -2 cos(k pi / (L + 1))."""
    from paper_0902_3185_amd import driver as DR
    L = 64
    log = DR.run(DR.hubbard(0.0), L, 512, 0, _init, ctx=ctx, prec="fp32", tol=1e-9)
    k = np.arange(1, L // 2 + 1)
    exact = 2 * np.sum(-2 * np.cos(k * np.pi / (L + 1)))
    e = log[-1]["energy"]
    assert log[-1]["n"] == L
    assert e >= exact - 1e-9 * L
    assert (e - exact) / L <= 1e-6, (e, exact)


def _dense_W(basis_dim, W):
    """Kept vectors {sector: dim x k} of a block with the given sector sizes,
    as one dense matrix (rows: the block's states; columns: kept states,
    sector by sector)."""
    off = np.concatenate([[0], np.cumsum(basis_dim)]).astype(int)
    secs = sorted(W)
    out = np.zeros((int(off[-1]), sum(W[s].shape[1] for s in secs)))
    c = 0
    for s in secs:
        out[off[s]:off[s + 1], c:c + W[s].shape[1]] = W[s]
        c += W[s].shape[1]
    return out


def _states(basis):
    from types import SimpleNamespace
    q = np.repeat(np.asarray(basis.q, dtype=np.int64), np.asarray(basis.dim, dtype=np.int64))
    return SimpleNamespace(n=len(q), q=q)


@pytest.mark.parametrize("name,L,m", [("hubbard_u4", 6, 4096), ("heisenberg", 16, 32)])
def test_carried_vector_matches_oracle_transformation(ctx, name, L, m):
    """Every start vector the GPU carries between finite-sweep steps equals,
    entry by entry, the oracle's wave-function transformation
    (carry_left_to_right / carry_right_to_left) applied to the GPU run's own
    ground state and kept vectors (both directions).  On the untruncated
    Hubbard chain each carried vector is also the next ground state
    (overlap >= 1 - 1e-10)."""
    from paper_0902_3185_amd import driver as DR
    model = DR.hubbard(4.0) if name == "hubbard_u4" else DR.heisenberg(DR.chain(1.0))
    Q = L + 1
    nu, nd = model.target(L)
    qt = int(nu + Q * nd)
    site_q = np.asarray(DR.site_block(model, 0, Q).basis.q, dtype=np.int64)
    seen, pending = [], []

    def on_carry(info):
        pending.append(dict(info, psi_old=info["psi_old"].cpu().numpy(), carried=info["carried"].cpu().numpy()))

    def on_solve(Sp, Ep, n, desc, r):
        if pending:
            c = pending.pop()
            c["psi_new"] = r["psi"].cpu().numpy()
            seen.append(c)

    DR.run(model, L, m, 1, _init, ctx=ctx, prec="fp64", tol=1e-12, on_carry=on_carry, on_solve=on_solve)
    assert len(seen) >= L - 4, len(seen)
    untruncated = name == "hubbard_u4"
    for c in seen:
        (So, Eo), (Sn, En) = c["old"], c["new"]
        sb_old = dict(S=dict(q=So.q, dim=So.dim), E=dict(q=Eo.q, dim=Eo.dim), q_target=qt)
        sb_new = dict(S=dict(q=Sn.q, dim=Sn.dim), E=dict(q=En.q, dim=En.dim), q_target=qt)
        other = _states(c["other"].basis)
        prod, kept = c["other"].origin
        other.W = _dense_W(prod.basis.dim, dict(kept) if isinstance(kept, list) else kept)
        trunc = _states(c["truncated"].basis)
        if c["direction"] == "left_to_right":
            W = _dense_W(So.dim, c["W"])
            ref = OD.carry_left_to_right(sb_old, c["psi_old"], W, trunc, other, site_q, sb_new)
        else:
            W = _dense_W(Eo.dim, c["W"])
            ref = OD.carry_right_to_left(sb_old, c["psi_old"], W, trunc, other, site_q, sb_new)
        got = c["carried"]
        assert got.shape == ref.shape
        assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref))), (c["direction"], c["p"])
        if untruncated:
            ov = abs(float(np.dot(got, c["psi_new"]))) / np.linalg.norm(got)
            assert ov >= 1 - 1e-10, (c["p"], ov)


def test_checkpoint_resume(ctx, tmp_path):
    """A run stopped after twelve steps (inside the first finite sweep) with
    checkpoints, then resumed from them, gives the uninterrupted run's steps
    and energies (to the solver's tolerance: the resumed run's steps start
    from carried vectors again); the superblock fixture written at the stop
    rebuilds that step's superblock, of which the saved vector is the ground
    state."""
    import torch
    from paper_0902_3185_amd import checkpoint as CK
    from paper_0902_3185_amd import driver as DR
    from paper_0902_3185_amd.superblock import Superblock
    L = 16
    model = DR.heisenberg(DR.chain(1.0))
    full = DR.run(model, L, 32, 2, _init, ctx=ctx, prec="fp64", tol=1e-10)
    pre = str(tmp_path / "run")
    part = DR.run(model, L, 32, 2, _init, ctx=ctx, prec="fp64", tol=1e-10, checkpoint=pre, stop_after=12)
    assert len(part) == 12
    for a, b in zip(part, full):
        assert a["energy"] == b["energy"]
    desc, psi = CK.load_superblock(pre + ".superblock.npz")
    sb = Superblock(desc, prec="fp64", ctx=ctx)
    r = sb.lanczos(torch.tensor(psi, dtype=torch.float64, device="cuda"), max_iter=50, tol=1e-9)
    assert r["iters"] == 1 and abs(r["energy"] - part[-1]["energy"]) <= 1e-12 * L
    rest = DR.run(model, L, 32, 2, _init, ctx=ctx, prec="fp64", tol=1e-10, checkpoint=pre, resume=pre)
    assert len(rest) == len(full)
    for a, b in zip(rest, full):
        assert (a["phase"], a["n"], a["p"]) == (b["phase"], b["n"], b["p"])
        assert abs(a["energy"] - b["energy"]) <= 1e-9 * L, (a, b)
    with pytest.raises(ValueError):
        DR.run(model, L, 16, 2, _init, ctx=ctx, prec="fp64", resume=pre)
