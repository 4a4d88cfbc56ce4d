"""Local density of states, Eq. (5) (oracle; test infrastructure).

N_i(omega) = int dt <psi| e^{-iHt} c^dag_i e^{iHt} c_i e^{i omega t} |psi>
           = 2 pi sum_n |<n|c_i|psi>|^2 delta(omega - (E0 - E_n)),
with |n>, E_n the eigenstates of H with one electron less.  The delta
function is broadened into a unit-area Lorentzian of half-width eta.
Two evaluations: the Lehmann sum over a full diagonalisation, and the
continued fraction of the Lanczos recursion started from c_i|psi>
(the paper's continued-fraction method).
"""
from __future__ import annotations

import numpy as np

from .models import _configs, _popcount, hubbard_sector_matrix


def lorentzian(x, eta):
    return eta / np.pi / (x * x + eta * eta)


def annihilator_bits(L, n_up, n_dn, site, spin):
    """c_{site, spin} from the (n_up, n_dn) to the reduced sector, in the
    bit-string basis of models.hubbard_sector_matrix (all up orbitals before
    all down orbitals, each ordered by site)."""
    cu, cd = _configs(L, n_up), _configs(L, n_dn)
    if spin == 0:
        cu2, cd2 = _configs(L, n_up - 1), cd
    else:
        cu2, cd2 = cu, _configs(L, n_dn - 1)
    M = np.zeros((len(cu2) * len(cd2), len(cu) * len(cd)))
    below = (1 << site) - 1
    for a, u in enumerate(cu):
        for b, d in enumerate(cd):
            if spin == 0:
                if not (u >> site) & 1:
                    continue
                sign = -1.0 if _popcount(np.array([u & below]))[0] % 2 else 1.0
                a2 = int(np.searchsorted(cu2, u ^ (1 << site)))
                M[a2 * len(cd2) + b, a * len(cd) + b] = sign
            else:
                if not (d >> site) & 1:
                    continue
                n_before = n_up + int(_popcount(np.array([d & below]))[0])
                sign = -1.0 if n_before % 2 else 1.0
                b2 = int(np.searchsorted(cd2, d ^ (1 << site)))
                M[a * len(cd2) + b2, a * len(cd) + b] = sign
    return M


def hubbard_ldos_lehmann(L, bonds, U, site, spin, omega, eta):
    """(N_i(omega), E0, weights, poles) of the half-filled Hubbard chain by ED."""
    n = L // 2
    H = hubbard_sector_matrix(L, bonds, U, n, n).toarray()
    w0, V0 = np.linalg.eigh(H)
    e0, psi = w0[0], V0[:, 0]
    nu2, nd2 = (n - 1, n) if spin == 0 else (n, n - 1)
    H2 = hubbard_sector_matrix(L, bonds, U, nu2, nd2).toarray()
    w, V = np.linalg.eigh(H2)
    amp = V.T @ (annihilator_bits(L, n, n, site, spin) @ psi)
    weights = amp * amp
    poles = e0 - w
    N = np.array([2 * np.pi * np.sum(weights * lorentzian(om - poles, eta)) for om in omega])
    return N, e0, weights, poles


def lanczos_coefficients(matvec, v0, nsteps):
    """(alpha, beta, ||v0||) of the Lanczos recursion from v0 with full
    reorthogonalisation; stops early when the Krylov space closes."""
    nrm = float(np.linalg.norm(v0))
    V = [v0 / nrm]
    alpha, beta = [], []
    for j in range(nsteps):
        w = matvec(V[-1])
        Vm = np.array(V).T
        for _ in range(2):
            w = w - Vm @ (Vm.T @ w)
        a = float(np.dot(V[-1], matvec(V[-1])))
        b = float(np.linalg.norm(w))
        alpha.append(a)
        beta.append(b)
        if b <= 1e-13 * max(1.0, abs(a)):
            break
        V.append(w / b)
    return np.array(alpha), np.array(beta), nrm


def ldos_continued_fraction(alpha, beta, weight, e0, omega, eta):
    """2 weight Im f(E0 - omega - i eta), f(z) = 1/(z - a0 - b0^2/(z - a1 - ...))."""
    out = []
    for om in omega:
        z = complex(e0 - om, -eta)
        f = 0.0
        for j in range(len(alpha) - 1, -1, -1):
            b2 = beta[j] ** 2 if j + 1 < len(alpha) else 0.0
            f = 1.0 / (z - alpha[j] - b2 * f)
        out.append(2 * weight * f.imag)
    return np.array(out)
