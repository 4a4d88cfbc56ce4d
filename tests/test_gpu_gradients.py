"""Coupling derivatives of the ground energy through the library (GPU).

H(J) = sum_g J_g H_g, every term of coupling group g being linear in J_g
(c_k = J_g * base_k for a bond term; the group's block-Hamiltonian term
carries J_g inside its operator).  So dE/dJ_g = <psi|H_g|psi> / J_g at the
ground state (Hellmann-Feynman), = sum over the group's terms of
(c_k / J_g) <psi|A_k (x) B_k|psi>, the adjoint's grad_c.  These tests check
that value three ways: against central finite differences of the Lanczos
ground energy, against the oracle's adjoint, and at the Majumdar-Ghosh
point where the exact answer is known.
"""
import numpy as np
import pytest

from oracle import superblock as OS
from workloads import init_vector, seeded_vector, workload_superblock

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_0902_3185_amd.superblock import Context
    return Context(0)


def _dev(x):
    import torch
    return torch.tensor(np.asarray(x), dtype=torch.float64, device="cuda")


def _group_scales(desc, J):
    """base_k = c_k / J_g of every term (the derivative of c_k by its group's coupling)."""
    return np.array([t["c"] / J[t["group"]] for t in desc["terms"]])


@pytest.mark.parametrize("m", [48, None])
def test_finite_difference_of_ground_energy(ctx, m):
    """Central differences (h = 1e-4) of the FP64 Lanczos ground energy by
    each coupling, against autograd's dE/dc combined per group; the same
    derivative from the oracle's adjoint at the GPU ground state."""
    import torch
    from paper_0902_3185_amd.autograd import hpsi
    from paper_0902_3185_amd.superblock import Superblock
    desc = workload_superblock("j1j2_L64_m256", m=m, seed=6)
    J = np.array(desc["meta"]["couplings"], dtype=float)
    base = _group_scales(desc, J)
    groups = np.array([t["group"] for t in desc["terms"]])
    sb = Superblock(desc, prec="fp64", ctx=ctx)
    psi0 = _dev(seeded_vector(sb.D, 61))
    print(f"j1j2 m={m} D={sb.D}", flush=True)

    def energy(Jv):
        sb.set_coeffs(base * Jv[groups])
        return sb.lanczos(psi0, max_iter=3000, tol=1e-11)

    r = energy(J)
    psi = r["psi"] / torch.linalg.vector_norm(r["psi"])
    c = torch.tensor(base * J[groups], dtype=torch.float64, requires_grad=True)
    E = torch.dot(psi, hpsi(psi, c, sb))
    E.backward()
    dEdc = c.grad.numpy()
    assert abs(E.item() - r["energy"]) <= 1e-12 * abs(r["energy"])
    _, gc_ref = OS.hpsi_adjoint_blocks(desc, psi.cpu().numpy(), psi.cpu().numpy())
    h = 1e-4
    for g in range(len(J)):
        sel = groups == g
        auto = float(np.sum(base[sel] * dEdc[sel]))
        orac = float(np.sum(base[sel] * gc_ref[sel]))
        Jp, Jm = J.copy(), J.copy()
        Jp[g] += h
        Jm[g] -= h
        fd = (energy(Jp)["energy"] - energy(Jm)["energy"]) / (2 * h)
        print(f"  group {g}: autograd {auto:.12f} oracle adjoint {orac:.12f} fd {fd:.12f}", flush=True)
        assert abs(auto - orac) <= 1e-10 * max(1.0, abs(orac))
        assert abs(auto - fd) <= 1e-6 * max(abs(fd), 1e-3 * abs(r["energy"])), (g, auto, fd)
    sb.set_coeffs(base * J[groups])


def test_majumdar_ghosh_derivatives(ctx):
    """J1-J2 chain at J2 = J1/2, L = 64, m = 256, one sweep on the GPU: the
    dimer state is exact, so every step gives E = -3n/8, and on the final
    superblock dE/dJ1 = <sum S_i.S_i+1> = -3L/8 = -24 and dE/dJ2 = 0
    through the adjoint."""
    import time
    from paper_0902_3185_amd import driver as DR
    from paper_0902_3185_amd.superblock import Superblock
    L, m = 64, 256
    last = {}

    def keep(Sp, Ep, n, desc, r):
        last.update(desc=desc, psi=r["psi"].clone())

    t0 = time.perf_counter()
    log = DR.run(DR.heisenberg(DR.j1j2(1.0, 0.5)), L, m, 1, lambda D, s: init_vector(D, s),
                 ctx=ctx, prec="fp32", tol=1e-9, on_solve=keep)
    print(f"Majumdar-Ghosh L={L} m={m}: {len(log)} steps in {time.perf_counter() - t0:.1f} s",
          flush=True)
    for r in log:
        assert abs(r["energy"] + 3 * r["n"] / 8) <= 1e-9 * r["n"], r
    desc = last["desc"]
    J = {0: 1.0, 1: 0.5}
    sb = Superblock(desc, prec="fp64", ctx=ctx)
    import torch
    psi = last["psi"] / torch.linalg.vector_norm(last["psi"])
    _, gc = sb.adjoint(psi, psi, want_psi=False, want_c=True)
    c = np.array([t["c"] for t in desc["terms"]])
    groups = np.array([t["group"] for t in desc["terms"]])
    d = {g: float(np.sum(c[groups == g] * np.asarray(gc)[groups == g])) / J[g] for g in (0, 1)}
    print(f"  dE/dJ1 = {d[0]:.12f}  dE/dJ2 = {d[1]:.3e}", flush=True)
    assert abs(d[0] + 3 * L / 8) <= 1e-7 * L
    assert abs(d[1]) <= 1e-7 * L
