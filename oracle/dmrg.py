"""Whole-run DMRG on dense block operators (oracle; test infrastructure).

Follows the paper's procedure (Sec. 1; the infinite loop of Sec. 3.1,
Fig. 2) step by step:

(a) grow the system: S' = S (x) X[step], the new site added on the right;
(b) grow the environment: E' = Y[step] (x) E, the new site added on the left;
    both rebuild the block Hamiltonian from the old one, the new site and the
    bonds between them (Sec. 3.3, setToProduct / addHamiltonianConnection),
    and reorder the product basis by increasing effective q (Sec. 3.2);
(c) the superblock S' (x) E' is a basis only -- its Hamiltonian is applied on
    the fly from the S' and E' operators (Sec. 3.3);
(d) its lowest state in the targeted symmetry sector, by Lanczos;
(e), (f) reduced density matrices (Eqs. (2), (3)), keep m states, change
    basis of the block Hamiltonian and operators (Eq. (4));
(g) store the block for the finite algorithm.

Block operators are plain dense matrices in the block's sorted basis; the
symmetry sectors are used only to restrict psi to the target and to
diagonalise rho sector by sector.

Readings where the paper is silent (its finite algorithm is "see code"):

* Infinite phase: the superblock of n sites is the open n-site system of
  the same model; S' covers positions 0..n/2-1 and E' the rest.  Left blocks
  label their sites by position, right blocks by distance from the right
  end, so a right block built for n sites is reused unchanged at larger n
  (all configurations here are translation invariant).
* Target: (N_up, N_down) = model.target(n) at every superblock size (half
  filling / S^z = 0).
* Finite phase: the superblock is split at p (S' = positions 0..p-1); one
  sweep goes p = L/2 -> L-2 truncating S', p = L-2 -> 2 truncating E', and
  p = 2 -> L/2 truncating S'.  The energy reported is the last one, at the
  centre.
* Fermion sign: a block carries its boundary-site operators with the
  Jordan-Wigner string through the block's sites to their left; the
  fermion parity F of a block is (-1)^(N_up + N_down), known from q.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .lanczos import lanczos_ground
from .rho import truncate
from .superblock import pack, target_indices, unpack


@dataclass
class Block:
    """A block with operators (DmrgBasisWithOperators, Sec. 3.3)."""
    sites: list            # labels: positions (left blocks) or distances from the right end
    q: np.ndarray          # effective quantum number per state, non-decreasing
    H: dict                # {coupling group: dense block Hamiltonian piece}
    ops: dict = field(default_factory=dict)   # {(label, name): dense operator}
    # kept eigenvectors (grown block's sorted basis x this block's states) when
    # the block was made by truncating a grown block; None for a bare site
    W: np.ndarray = None

    @property
    def n(self):
        return len(self.q)

    def H_total(self):
        return sum(self.H.values())


def sectors(q):
    """(distinct q values, their multiplicities) of a sorted q array (Sec. 3.2 partition)."""
    u, c = np.unique(q, return_counts=True)
    return dict(q=u.astype(np.int64), dim=c.astype(np.int64))


def parity(block, model, Q):
    """Fermion parity (-1)^N of every state, as a diagonal matrix."""
    if not model.fermionic:
        return np.eye(block.n)
    N = block.q % Q + block.q // Q
    return np.diag(np.where(N % 2 == 0, 1.0, -1.0))


def site_block(model, label, Q):
    """A one-site block in its natural basis (setNaturalBasis, Sec. 4.1), sorted by q."""
    q = model.q_site(Q)
    perm = np.argsort(q, kind="stable")
    ops = {(label, name): model.site[name][np.ix_(perm, perm)] for name in model.carried}
    return Block(sites=[label], q=q[perm], H={-1: model.onsite[np.ix_(perm, perm)]}, ops=ops)


def _op(block, label, name, transpose):
    M = block.ops[(label, name)]
    return M.T if transpose else M


def _sorted(block_q, H, ops, sites):
    perm = np.argsort(block_q, kind="stable")
    P = np.ix_(perm, perm)
    return Block(sites=sites, q=block_q[perm],
                 H={g: h[P] for g, h in H.items()},
                 ops={k: o[P] for k, o in ops.items()})


def bond_terms(model, left, right, F_left, lab_left, lab_right, value):
    """[(coefficient, left operator, right operator)] of one bond between two parts."""
    out = []
    for (f, ln, lt, rn, rt, fm) in model.bond_ops:
        A = _op(left, lab_left, ln, lt)
        if fm == "OF":
            A = A @ F_left
        elif fm == "FO":
            A = F_left @ A
        out.append((value * f, A, _op(right, lab_right, rn, rt)))
    return out


def _add(H, g, M):
    H[g] = H[g] + M if g in H else M


def grow_right(S, model, Q, bonds, keep_range):
    """S' = S (x) x with x the next position (Fig. 2(a), GROW_RIGHT)."""
    x = max(S.sites) + 1
    site = site_block(model, x, Q)
    d, NS = site.n, S.n
    IS, Id = np.eye(NS), np.eye(d)
    H = {}
    for g, h in S.H.items():
        _add(H, g, np.kron(h, Id))
    for g, h in site.H.items():
        _add(H, g, np.kron(IS, h))
    FS = parity(S, model, Q)
    for (i, j, v, g) in bonds:
        if j == x and i in S.sites:
            for (c, A, B) in bond_terms(model, S, site, FS, i, x, v):
                _add(H, g, c * np.kron(A, B))
    ops = {}
    for (lab, name), O in S.ops.items():
        if lab > x - keep_range:
            ops[(lab, name)] = np.kron(O, Id)
    for (lab, name), o in site.ops.items():
        ops[(lab, name)] = np.kron(FS if model.fermionic else IS, o)
    q = (S.q[:, None] + site.q[None, :]).reshape(-1)
    return _sorted(q, H, ops, S.sites + [x])


def grow_left(E, model, Q, n, bonds, keep_range):
    """E' = y (x) E with y the next site to the left (Fig. 2(b), GROW_LEFT).

    Right-block labels are distances from the right end of the n-site system.
    """
    r = max(E.sites) + 1
    site = site_block(model, r, Q)
    d, NE = site.n, E.n
    IE, Id = np.eye(NE), np.eye(d)
    H = {}
    for g, h in site.H.items():
        _add(H, g, np.kron(h, IE))
    for g, h in E.H.items():
        _add(H, g, np.kron(Id, h))
    Fy = parity(site, model, Q)
    py = n - 1 - r
    for (i, j, v, g) in bonds:
        if i == py and (n - 1 - j) in E.sites:
            for (c, A, B) in bond_terms(model, site, E, Fy, r, n - 1 - j, v):
                _add(H, g, c * np.kron(A, B))
    ops = {}
    for (lab, name), o in site.ops.items():
        ops[(lab, name)] = np.kron(o, IE)
    for (lab, name), O in E.ops.items():
        if lab > r - keep_range:
            ops[(lab, name)] = np.kron(Fy if model.fermionic else Id, O)
    q = (site.q[:, None] + E.q[None, :]).reshape(-1)
    return _sorted(q, H, ops, E.sites + [r])


def superblock_terms(Sp, Ep, model, Q, n, bonds):
    """Dense terms (c, A on S', B on E', group) of H_{S' u E'} (Sec. 3.3).

    H_S' (x) I and I (x) H_E' per coupling group, then every bond between a
    site of S' (positions) and a site of E' (labels n-1-position).
    """
    terms = []
    for g, h in sorted(Sp.H.items()):
        terms.append((1.0, h, None, g))
    for g, h in sorted(Ep.H.items()):
        terms.append((1.0, None, h, g))
    FS = parity(Sp, model, Q)
    for (i, j, v, g) in bonds:
        if i in Sp.sites and (n - 1 - j) in Ep.sites:
            for (c, A, B) in bond_terms(model, Sp, Ep, FS, i, n - 1 - j, v):
                terms.append((c, A, B, g))
    return terms


def describe(Sp, Ep, terms, q_target):
    """The superblock as block-sparse data (the format of ``superblock``)."""
    S, E = sectors(Sp.q), sectors(Ep.q)

    def blocks(M, basis):
        if M is None:
            return None
        o = np.concatenate([[0], np.cumsum(basis["dim"])])
        out, deltas = [], set()
        for r in range(len(basis["q"])):
            for c in range(len(basis["q"])):
                blk = M[o[r]:o[r + 1], o[c]:o[c + 1]]
                if np.any(blk != 0.0):
                    out.append((r, c, blk.copy()))
                    deltas.add(int(basis["q"][r] - basis["q"][c]))
        if len(deltas) > 1:
            raise ValueError("operator mixes quantum-number shifts")
        return dict(delta=deltas.pop() if deltas else 0, blocks=out)

    return dict(S=S, E=E, q_target=int(q_target),
                terms=[dict(c=c, A=blocks(A, S), B=blocks(B, E), group=g)
                       for (c, A, B, g) in terms])


def superblock_matvec(sb, terms):
    """psi -> H psi on the target sector, H = sum of c A (x) B (Sec. 3.3)."""
    def matvec(psi):
        P = unpack(sb, psi)
        Y = np.zeros_like(P)
        for (c, A, B, _g) in terms:
            T = P if A is None else A @ P
            T = T if B is None else T @ B.T
            Y += c * T
        return pack(sb, Y)
    return matvec


def solve(Sp, Ep, terms, q_target, init, tol, max_iter):
    """Lowest state of the superblock in the target sector (Fig. 2(d)).

    ``init(D)`` gives the Lanczos start vector."""
    sb = dict(S=sectors(Sp.q), E=sectors(Ep.q), q_target=int(q_target))
    D = len(target_indices(sb))
    E0, psi, it, res = lanczos_ground(superblock_matvec(sb, terms), init(D),
                                      max_iter=max_iter, tol=tol)
    return sb, E0, psi, it, res


def change_basis(block, sb, psi, side, m, no_split):
    """Truncate a grown block with its density matrix (Fig. 2(e)/(f), Eq. (4))."""
    tr = truncate(sb, psi, side, m, no_split=no_split)
    basis = sb["S"] if side == 0 else sb["E"]
    o = np.concatenate([[0], np.cumsum(basis["dim"])])
    cols, qs = [], []
    for s in sorted(tr["W"].keys()):
        Ws = tr["W"][s]
        full = np.zeros((block.n, Ws.shape[1]))
        full[o[s]:o[s + 1], :] = Ws
        cols.append(full)
        qs += [int(basis["q"][s])] * Ws.shape[1]
    W = np.hstack(cols)
    new = Block(sites=list(block.sites), q=np.array(qs, dtype=np.int64),
                H={g: W.T @ h @ W for g, h in block.H.items()},
                ops={k: W.T @ O @ W for k, O in block.ops.items()}, W=W)
    return new, tr


# ---------------------------------------------------------------------------
# Wave-function transformation (the paper's conclusions name it, after White,
# as what makes a good Lanczos start vector in the finite phase).  The paper
# gives no formula; the reading used is the plain change of basis of the
# state, written out on dense matrices:
#
#   split p -> p+1 (S' was truncated at p):  Psi(p) is a matrix over
#   S'(p) x E'(p), E'(p) = site(p+1) (x) R with R = R_{L-p-1}, itself the
#   truncation W_R of E'(p+1) = site(p+2) (x) R_{L-p-2}.  Then
#       Psi(p+1)[(a, s), e'] = sum_{alpha, r} W_L[alpha, a] Psi(p)[alpha, (s, r)] W_R[e', r]
#   with a a state of the truncated S(p), s the state of site p+1, and
#   (a, s) placed in the sorted basis of S'(p+1) = S(p) (x) site(p+1).
#   split p -> p-1 is the mirror image, with the roles of the blocks swapped.
#
# Untruncated, both maps are exact changes of basis of the same L-site
# state: the carried vector is then the next step's ground state itself.
# ---------------------------------------------------------------------------


def product_order(q_major, q_minor):
    """Sort permutation of the product basis (major index outer), the same
    stable ordering by effective q that grow_right / grow_left apply (Sec. 3.2):
    sorted state k is product state perm[k]."""
    q = (np.asarray(q_major)[:, None] + np.asarray(q_minor)[None, :]).reshape(-1)
    return np.argsort(q, kind="stable")


def carry_left_to_right(sb_old, psi, W_L, S_new, R_old, site_q, sb_new):
    """Start vector at split p+1 from the ground state psi at split p.

    W_L: kept vectors of S'(p) (the truncation just made), S_new = S(p);
    R_old = R_{L-p-1} with R_old.W its kept vectors in the sorted basis of
    E'(p+1) = site (x) R_{L-p-2}; site_q: one site's sorted q."""
    Psi = unpack(sb_old, psi)                          # S'(p) x E'(p), sorted
    d, nR = len(site_q), R_old.n
    permE = product_order(site_q, R_old.q)             # E'(p) = site (x) R_old
    U = np.zeros_like(Psi)
    U[:, permE] = Psi                                  # columns in product order (s, r)
    U = U.reshape(Psi.shape[0], d, nR)
    T = np.einsum("xa,xsr,er->ase", W_L, U, R_old.W)   # (a, s, e') ; e' in E'(p+1)
    T = T.reshape(S_new.n * d, R_old.W.shape[0])       # rows in product order (a, s)
    permS = product_order(S_new.q, site_q)             # S'(p+1) = S(p) (x) site
    return pack(sb_new, T[permS, :])


def carry_right_to_left(sb_old, psi, W_E, E_new, L_old, site_q, sb_new):
    """Start vector at split p-1 from the ground state psi at split p.

    W_E: kept vectors of E'(p) (the truncation just made), E_new = E(p);
    L_old = S_{p-1} with L_old.W its kept vectors in the sorted basis of
    S'(p-1) = S_{p-2} (x) site; site_q: one site's sorted q."""
    Psi = unpack(sb_old, psi)                          # S'(p) x E'(p), sorted
    d, nL = len(site_q), L_old.n
    permS = product_order(L_old.q, site_q)             # S'(p) = L_old (x) site
    U = np.zeros_like(Psi)
    U[permS, :] = Psi                                  # rows in product order (l, s)
    U = U.reshape(nL, d, Psi.shape[1])
    T = np.einsum("al,lsy,ye->ase", L_old.W, U, W_E)   # (a', s, e) ; a' in S'(p-1)
    T = T.reshape(L_old.W.shape[0], d * E_new.n)       # columns in product order (s, e)
    permE = product_order(site_q, E_new.q)             # E'(p-1) = site (x) E(p)
    return pack(sb_new, T[:, permE])


def _q_target(model, n, Q):
    nu, nd = model.target(n)
    return nu + Q * nd


def run(model, L, m, sweeps, init, tol=1e-10, max_iter=300, no_split=True,
        keep_range=None, on_superblock=None, wavefunction=False):
    """Infinite phase to L sites, then ``sweeps`` finite sweeps.

    ``init(D, step)`` supplies the Lanczos initial vector of each step (an
    input, so that both sides of a comparison can use the same one).  In the
    finite phase the previous ground state is also carried to the new basis
    (carry_left_to_right / carry_right_to_left; unchanged when the split
    stays put); its record gets ``carry_overlap`` = |<carried|psi>| / |carried|
    against the new ground state and ``carry_energy`` = its Rayleigh quotient.
    With ``wavefunction`` set, the carried vector is the Lanczos start.
    Returns a list of per-step records (dicts).
    """
    Q = L + 1
    if keep_range is None:
        keep_range = max(j - i for (i, j, _v, _g) in model.bonds(L))
    log = []
    step = 0
    left = {1: site_block(model, 0, Q)}
    right = {1: site_block(model, 0, Q)}
    site_q = left[1].q
    prev = {}

    def carried(p, sb_new):
        """The previous ground state in the basis of the superblock at split p."""
        if not prev or prev["n"] != L:
            return None
        if prev["p"] == p:
            return prev["psi"]
        if prev["p"] + 1 == p and 0 in prev["out"]:
            return carry_left_to_right(prev["sb"], prev["psi"], prev["out"][0].W,
                                       prev["out"][0], right[L - p], site_q, sb_new)
        if prev["p"] - 1 == p and 1 in prev["out"]:
            return carry_right_to_left(prev["sb"], prev["psi"], prev["out"][1].W,
                                       prev["out"][1], left[p], site_q, sb_new)
        return None

    def one(Sp, Ep, n, truncate_sides, phase, p):
        nonlocal step
        bonds = model.bonds(n)
        terms = superblock_terms(Sp, Ep, model, Q, n, bonds)
        qt = _q_target(model, n, Q)
        if on_superblock is not None:
            on_superblock(phase, n, p, describe(Sp, Ep, terms, qt))
        sb0 = dict(S=sectors(Sp.q), E=sectors(Ep.q), q_target=int(qt))
        c = carried(p, sb0) if phase == "finite" else None
        start = (lambda D: c) if (wavefunction and c is not None
                                  and np.linalg.norm(c) > 0.0) else (lambda D: init(D, step))
        sb, E0, psi, it, res = solve(Sp, Ep, terms, qt, start, tol, max_iter)
        rec = dict(phase=phase, n=n, p=p, energy=E0, iters=it, resid=res,
                   dimS=Sp.n, dimE=Ep.n, D=len(psi), step=step)
        if c is not None and np.linalg.norm(c) > 0.0:
            nc = float(np.linalg.norm(c))
            rec["carry_overlap"] = abs(float(np.dot(c, psi))) / nc
            rec["carry_energy"] = float(np.dot(c, superblock_matvec(sb, terms)(c))) / nc ** 2
        out = {}
        for side in truncate_sides:
            blk = Sp if side == 0 else Ep
            new, tr = change_basis(blk, sb, psi, side, m, no_split)
            rec["eps%d" % side] = tr["eps"]
            rec["straddle%d" % side] = tr["straddle"]
            out[side] = new
        log.append(rec)
        step += 1
        prev.clear()
        prev.update(n=n, p=p, sb=sb, psi=psi, out=out)
        return out

    # infinite phase (Fig. 2): superblocks of n = 4, 6, ..., L sites
    for n in range(4, L + 1, 2):
        h = n // 2
        bonds = model.bonds(n)
        Sp = grow_right(left[h - 1], model, Q, bonds, keep_range)
        Ep = grow_left(right[h - 1], model, Q, n, bonds, keep_range)
        out = one(Sp, Ep, n, (0, 1), "infinite", h)
        left[h], right[h] = out[0], out[1]

    # finite sweeps (Sec. 1)
    bonds = model.bonds(L)
    for _ in range(sweeps):
        path = ([(p, 0) for p in range(L // 2, L - 1)]
                + [(p, 1) for p in range(L - 2, 1, -1)]
                + [(p, 0) for p in range(2, L // 2 + 1)])
        for (p, side) in path:
            Sp = grow_right(left[p - 1], model, Q, bonds, keep_range)
            Ep = grow_left(right[L - p - 1], model, Q, L, bonds, keep_range)
            out = one(Sp, Ep, L, (side,), "finite", p)
            if side == 0:
                left[p] = out[0]
            else:
                right[L - p] = out[1]
    return log
