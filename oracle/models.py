"""Models, geometries and exact diagonalisation (oracle; test infrastructure).

Follows the paper's Sec. 1 (one-site state sets C), Sec. 3.2 (effective
quantum number q = sum_a qt_a Q^a) and Sec. 4.1 (the Hubbard and spin-1/2
Heisenberg Hamiltonians), and Sec. 4.2 (chains and n-leg ladders).

Readings where the paper is silent:

* Fermion ordering: Jordan-Wigner by chain position, up before down inside a
  site, |up,down> = c^dag_up c^dag_down |e>.  (The exact diagonalisation below
  uses a different but equivalent ordering -- all up orbitals before all down
  orbitals -- so the two can pin each other.)
* The hopping sum is taken once per bond plus its Hermitian conjugate,
  t (c^dag_i c_j + c^dag_j c_i); on bipartite open chains the sign of t is a
  gauge choice.
* The Hubbard interaction is U n_up n_down (no half-filling shift).
* Ladder sites are numbered rung by rung ("snake"): site = 2 x + y.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from itertools import combinations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


# ---------------------------------------------------------------------------
# One-site operators (Sec. 1: C = {up, down} for spin-1/2,
# C = {e, up, down, (up,down)} for Hubbard; Sec. 3.3: c_{i sigma} and
# S^+_i, S^z_i are the operators each model keeps).
# ---------------------------------------------------------------------------

def spin_half_site():
    """Spin-1/2 site in the order (up, down).

    Returns the site dimension, S^z, S^+, S^- and the number of up spins per
    state, which is the (only) conserved quantity used for spin models.
    """
    sz = np.diag([0.5, -0.5])
    sp_ = np.array([[0.0, 1.0], [0.0, 0.0]])  # |up><down|
    return dict(d=2, Sz=sz, Sp=sp_, Sm=sp_.T.copy(),
                nup=np.array([1, 0]), ndn=np.array([0, 0]))


def hubbard_site():
    """Hubbard site in the order (e, up, down, updown), Sec. 1.

    |updown> = c^dag_up c^dag_down |e>, so c_down |updown> = -|up> and
    c_up |updown> = +|down>.
    """
    c_up = np.zeros((4, 4))
    c_dn = np.zeros((4, 4))
    c_up[0, 1] = 1.0      # c_up |up> = |e>
    c_up[2, 3] = 1.0      # c_up |updown> = |down>
    c_dn[0, 2] = 1.0      # c_down |down> = |e>
    c_dn[1, 3] = -1.0     # c_down |updown> = -|up>
    n_up = c_up.T @ c_up
    n_dn = c_dn.T @ c_dn
    return dict(d=4, c_up=c_up, c_dn=c_dn, n_up=n_up, n_dn=n_dn,
                F=np.diag([1.0, -1.0, -1.0, 1.0]),
                nup=np.array([0, 1, 0, 1]), ndn=np.array([0, 0, 1, 1]))


# ---------------------------------------------------------------------------
# Geometries (Sec. 4.2): lists of bonds (i, j, value, group) with i < j.
# ``group`` labels the coupling a bond belongs to (J1 / J2, rung / leg) so
# that derivatives with respect to a coupling can be formed term by term.
# ---------------------------------------------------------------------------

def chain_bonds(L, value=1.0):
    """Open 1-D chain: nearest-neighbour bonds (DmrgGeometryOneD)."""
    return [(i, i + 1, float(value), 0) for i in range(L - 1)]


def j1j2_bonds(L, j1, j2):
    """Open chain with nearest (group 0) and next-nearest (group 1) bonds."""
    b = [(i, i + 1, float(j1), 0) for i in range(L - 1)]
    b += [(i, i + 2, float(j2), 1) for i in range(L - 2)]
    return sorted(b, key=lambda t: (t[0], t[1]))


def ladder_bonds(W, j_leg=1.0, j_rung=1.0):
    """Two-leg ladder of W rungs, sites numbered rung by rung (site = 2x+y).

    Rungs (2x, 2x+1) are group 0, legs (2x+y, 2x+2+y) group 1.
    """
    b = []
    for x in range(W):
        b.append((2 * x, 2 * x + 1, float(j_rung), 0))
        if x + 1 < W:
            for y in range(2):
                b.append((2 * x + y, 2 * x + 2 + y, float(j_leg), 1))
    return sorted(b, key=lambda t: (t[0], t[1]))


# ---------------------------------------------------------------------------
# Exact diagonalisation with bit strings (ground truth for the pins).
# ---------------------------------------------------------------------------

def _configs(L, n):
    """All L-bit integers with n bits set, ascending."""
    out = []
    for occ in combinations(range(L), n):
        v = 0
        for i in occ:
            v |= 1 << i
        out.append(v)
    return np.array(sorted(out), dtype=np.int64)


def _popcount(a):
    a = np.asarray(a, dtype=np.int64)
    c = np.zeros_like(a)
    x = a.copy()
    while np.any(x):
        c += x & 1
        x >>= 1
    return c


def _lowest(H, k=1):
    n = H.shape[0]
    if n <= 2500:
        w, v = np.linalg.eigh(H.toarray() if sp.issparse(H) else H)
        return w[:k], v[:, :k]
    w, v = spla.eigsh(H, k=k, which="SA", tol=1e-13, maxiter=100000)
    order = np.argsort(w)
    return w[order], v[:, order]


def heisenberg_sector_matrix(L, bonds, n_up):
    """Spin-1/2 H = sum_bonds J S_i.S_j (Sec. 4.1) in the sector with n_up up spins.

    Bit i set means site i is up.  S_i.S_j = S^z S^z + (S^+S^- + S^-S^+)/2.
    """
    states = _configs(L, n_up)
    n = len(states)
    rows, cols, vals = [], [], []
    diag = np.zeros(n)
    for (i, j, J, _g) in bonds:
        bi = (states >> i) & 1
        bj = (states >> j) & 1
        same = bi == bj
        diag += np.where(same, 0.25 * J, -0.25 * J)
        flip = np.nonzero(~same)[0]
        new = states[flip] ^ ((1 << i) | (1 << j))
        idx = np.searchsorted(states, new)
        rows.append(idx)
        cols.append(flip)
        vals.append(np.full(len(flip), 0.5 * J))
    rows.append(np.arange(n))
    cols.append(np.arange(n))
    vals.append(diag)
    H = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    return H


def heisenberg_ed(L, bonds, n_up=None, k=1):
    """Lowest k energies of the spin-1/2 Heisenberg model in the n_up sector."""
    if n_up is None:
        n_up = L // 2
    w, _ = _lowest(heisenberg_sector_matrix(L, bonds, n_up), k)
    return w


def _hop_matrix(L, configs, bonds):
    """One-species hopping sum_bonds t (c^dag_i c_j + h.c.) on bit strings.

    Orbitals of one species are ordered by site; moving an electron between
    i and j picks up (-1)^(number of same-species electrons strictly
    between them).
    """
    n = len(configs)
    rows, cols, vals = [], [], []
    for (i, j, t, _g) in bonds:
        a, b = min(i, j), max(i, j)
        between = 0
        for s in range(a + 1, b):
            between |= 1 << s
        ba = (configs >> a) & 1
        bb = (configs >> b) & 1
        src = np.nonzero((bb == 1) & (ba == 0))[0]     # electron at b hops to a
        new = configs[src] ^ ((1 << a) | (1 << b))
        sign = np.where(_popcount(configs[src] & between) % 2 == 0, 1.0, -1.0)
        idx = np.searchsorted(configs, new)
        rows += [idx, src]
        cols += [src, idx]
        vals += [t * sign, t * sign]
    if not rows:
        return sp.csr_matrix((n, n))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))


def hubbard_sector_matrix(L, bonds, U, n_up, n_dn, V=0.0):
    """Hubbard H = sum t (c^dag c + h.c.) + sum U n_up n_dn + sum V n (Sec. 4.1).

    Basis: (up configuration, down configuration), index iu*n_dn_cfg + id.
    ``U`` and ``V`` may be scalars or per-site arrays.
    """
    U = np.broadcast_to(np.asarray(U, dtype=float), (L,))
    V = np.broadcast_to(np.asarray(V, dtype=float), (L,))
    cu = _configs(L, n_up)
    cd = _configs(L, n_dn)
    Tu = _hop_matrix(L, cu, bonds)
    Td = _hop_matrix(L, cd, bonds)
    H = sp.kron(Tu, sp.identity(len(cd))) + sp.kron(sp.identity(len(cu)), Td)
    diag = np.zeros(len(cu) * len(cd))
    uu = cu[:, None]
    dd = cd[None, :]
    for s in range(L):
        nu = ((uu >> s) & 1).astype(float)
        nd = ((dd >> s) & 1).astype(float)
        diag += (U[s] * nu * nd + V[s] * (nu + nd)).reshape(-1)
    return (H + sp.diags(diag)).tocsr()


def hubbard_ed(L, bonds, U, n_up=None, n_dn=None, V=0.0, k=1):
    """Lowest k energies of the Hubbard model in the (n_up, n_dn) sector."""
    if n_up is None:
        n_up = L // 2
    if n_dn is None:
        n_dn = L // 2
    w, _ = _lowest(hubbard_sector_matrix(L, bonds, U, n_up, n_dn, V), k)
    return w


# ---------------------------------------------------------------------------
# Full Fock-space operators by Kronecker products with Jordan-Wigner strings
# (the ordering the DMRG blocks use).  Small L only.
# ---------------------------------------------------------------------------

def fock_annihilators(L):
    """c_{i,sigma} on the 4^L Hubbard Fock space, JW ordered by site (up first)."""
    site = hubbard_site()
    F = sp.csr_matrix(site["F"])
    I = sp.identity(4, format="csr")
    out = []
    for i in range(L):
        ops = []
        for c in (site["c_up"], site["c_dn"]):
            m = sp.identity(1, format="csr")
            for s in range(L):
                f = F if s < i else (sp.csr_matrix(c) if s == i else I)
                m = sp.kron(m, f, format="csr")
            ops.append(m)
        out.append(ops)
    return out


def spin_operators(L):
    """S^z_i, S^+_i on the 2^L spin space by Kronecker products."""
    site = spin_half_site()
    I = sp.identity(2, format="csr")
    out = []
    for i in range(L):
        d = {}
        for name in ("Sz", "Sp"):
            m = sp.identity(1, format="csr")
            for s in range(L):
                m = sp.kron(m, sp.csr_matrix(site[name]) if s == i else I, format="csr")
            d[name] = m
        out.append(d)
    return out


def hubbard_fock_hamiltonian(L, bonds, U, V=0.0):
    """Hubbard H on the full Fock space built from JW-stringed c operators."""
    c = fock_annihilators(L)
    U = np.broadcast_to(np.asarray(U, dtype=float), (L,))
    V = np.broadcast_to(np.asarray(V, dtype=float), (L,))
    H = sp.csr_matrix((4 ** L, 4 ** L))
    for (i, j, t, _g) in bonds:
        for s in range(2):
            hop = c[i][s].T @ c[j][s]
            H = H + t * (hop + hop.T)
    for i in range(L):
        nu = c[i][0].T @ c[i][0]
        nd = c[i][1].T @ c[i][1]
        H = H + U[i] * (nu @ nd) + V[i] * (nu + nd)
    return H.tocsr()


def hubbard_fock_numbers(L):
    """(N_up, N_down) of every Fock basis state, in Kronecker order."""
    site = hubbard_site()
    nu = np.zeros(1, dtype=np.int64)
    nd = np.zeros(1, dtype=np.int64)
    for _ in range(L):
        nu = (nu[:, None] + site["nup"][None, :]).reshape(-1)
        nd = (nd[:, None] + site["ndn"][None, :]).reshape(-1)
    return nu, nd


def heisenberg_kron_hamiltonian(L, bonds):
    """Spin-1/2 H on the full 2^L space from Kronecker-product spin operators."""
    S = spin_operators(L)
    H = sp.csr_matrix((2 ** L, 2 ** L))
    for (i, j, J, _g) in bonds:
        H = H + J * (S[i]["Sz"] @ S[j]["Sz"]
                     + 0.5 * (S[i]["Sp"] @ S[j]["Sp"].T + S[i]["Sp"].T @ S[j]["Sp"]))
    return H.tocsr()


def spin_kron_nup(L):
    site = spin_half_site()
    n = np.zeros(1, dtype=np.int64)
    for _ in range(L):
        n = (n[:, None] + site["nup"][None, :]).reshape(-1)
    return n


# ---------------------------------------------------------------------------
# Model descriptions used by the oracle DMRG.
# ---------------------------------------------------------------------------

@dataclass
class Model:
    """A lattice model as the DMRG needs it (the DmrgModelBase interface, Sec. 4.1).

    ``site``       one-site operator dictionary (spin_half_site / hubbard_site)
    ``fermionic``  whether bond operators carry Jordan-Wigner parity
    ``onsite``     one-site Hamiltonian (d x d)
    ``carried``    names of the one-site operators a block keeps for each of
                   its boundary sites (Sec. 3.3: c_{i sigma}; S^+_i, S^z_i)
    ``bond_ops``   [(factor, left, left_T, right, right_T, fmode)]: a bond
                   (i < j) of value v contributes
                   v * factor * op(left)_i op(right)_j, where ``*_T`` asks for
                   the transpose (S^- = (S^+)^T, c^dag = c^T in a real basis)
                   and ``fmode`` places the left part's fermion parity F:
                   "OF" -> (O_i F) (x) O_j, "FO" -> (F O_i) (x) O_j, "" -> none.
    ``bonds``      function L -> list of bonds (i, j, value, group)
    ``target``     function n_sites -> (N_up, N_down) targeted by the superblock
    """
    name: str
    site: dict
    fermionic: bool
    onsite: np.ndarray
    carried: tuple
    bond_ops: list
    bonds: object
    target: object
    extra: dict = field(default_factory=dict)

    def q_site(self, Q):
        """Effective quantum number of each one-site state (Sec. 3.2)."""
        return self.site["nup"] + Q * self.site["ndn"]


def heisenberg_model(bond_fn):
    """Spin-1/2 Heisenberg sum J_ij S_i.S_j (Sec. 4.1); conserved: N_up (S^z)."""
    return Model(
        name="heisenberg", site=spin_half_site(), fermionic=False,
        onsite=np.zeros((2, 2)), carried=("Sz", "Sp"),
        bond_ops=[(1.0, "Sz", False, "Sz", False, ""),
                  (0.5, "Sp", False, "Sp", True, ""),
                  (0.5, "Sp", True, "Sp", False, "")],
        bonds=bond_fn,
        target=lambda n: (n // 2, 0))


def hubbard_model(U, t=1.0, V=0.0):
    """One-band Hubbard model (Sec. 4.1) on an open chain; conserved (N_up, N_down).

    t (c^dag_i c_j + c^dag_j c_i) with i in the left part and j in the right
    part becomes t (c^dag_i F) (x) c_j + t (F c_i) (x) c^dag_j, F being the
    fermion parity of the left part.
    """
    site = hubbard_site()
    onsite = U * (site["n_up"] @ site["n_dn"]) + V * (site["n_up"] + site["n_dn"])
    ops = []
    for s in ("c_up", "c_dn"):
        ops.append((1.0, s, True, s, False, "OF"))
        ops.append((1.0, s, False, s, True, "FO"))
    return Model(
        name="hubbard", site=site, fermionic=True, onsite=onsite,
        carried=("c_up", "c_dn"), bond_ops=ops,
        bonds=lambda L: chain_bonds(L, t),
        target=lambda n: (n // 2, n // 2),
        extra=dict(U=U, t=t, V=V))
