"""Whole-run DMRG on top of libdmrg: the infinite loop of the paper's
Sec. 3.1 (Fig. 2) and the finite sweeps of Sec. 1.

Host bookkeeping (the paper's ``grow`` / ``setToProduct``, Sec. 3.3) keeps
block operators block-sparse by effective quantum number (Sec. 3.2): a grown
block S' = S (x) x is a list of "runs" -- one per (S sector, site state) with
q_S + q_x fixed -- and every product operator A (x) a is assembled from
A's sector blocks scaled by a's entries, run by run.  Everything on the
superblock goes through the library: the product, the Lanczos ground state
(FP64, or FP32 products with FP64 cycles), the density-matrix truncation,
and the change of basis of the block Hamiltonian and carried operators
(Eq. (4)) on the GPU.

Readings (shared with the oracle, stated in the repository's design notes):
the infinite-phase superblock of n sites is the open n-site system; right
blocks label sites by distance from the right end; a finite sweep goes
p = L/2 -> L-2 (truncate S'), L-2 -> 2 (truncate E'), 2 -> L/2; fermion
signs by Jordan-Wigner order with the left part's parity on bond terms.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

DEVICE = "cuda"   # where the driver keeps psi and staging buffers

# ---------------------------------------------------------------------------
# Models (Sec. 4.1) and geometries (Sec. 4.2)
# ---------------------------------------------------------------------------


@dataclass
class SiteModel:
    """One-site basis and operators of a model, states in increasing q."""
    name: str
    qsite: object            # function Q -> effective q of each state
    parity: np.ndarray       # +1 / -1 fermion parity per state (all +1 for spins)
    onsite: np.ndarray       # d x d one-site Hamiltonian
    ops: dict                # carried one-site operators, name -> d x d
    bond: list               # [(factor, left, left_T, right, right_T, fmode)]
    bonds: object            # L -> [(i, j, value, group)]
    target: object           # n -> (N_up, N_down)
    fermionic: bool = False

    @property
    def d(self):
        return self.onsite.shape[0]


def heisenberg(bonds):
    """Spin-1/2 sum J S_i.S_j; states (down, up), q = N_up."""
    sz = np.diag([-0.5, 0.5])
    spl = np.array([[0.0, 0.0], [1.0, 0.0]])      # S+|down> = |up>
    return SiteModel(
        name="heisenberg", qsite=lambda Q: np.array([0, 1]), parity=np.ones(2),
        onsite=np.zeros((2, 2)), ops={"Sz": sz, "Sp": spl},
        bond=[(1.0, "Sz", False, "Sz", False, ""), (0.5, "Sp", False, "Sp", True, ""),
              (0.5, "Sp", True, "Sp", False, "")],
        bonds=bonds, target=lambda n: (n // 2, 0))


def hubbard(U, t=1.0):
    """Hubbard t (c^dag c + h.c.) + U n_up n_dn; states (e, up, down, updown)
    with q = N_up + Q N_down, |updown> = c^dag_up c^dag_down |e>."""
    cu = np.zeros((4, 4))
    cd = np.zeros((4, 4))
    cu[0, 1] = cu[2, 3] = 1.0
    cd[0, 2] = 1.0
    cd[1, 3] = -1.0
    nu, nd = cu.T @ cu, cd.T @ cd
    bond = []
    for s in ("cu", "cd"):
        bond.append((1.0, s, True, s, False, "OF"))
        bond.append((1.0, s, False, s, True, "FO"))
    return SiteModel(
        name="hubbard", qsite=lambda Q: np.array([0, 1, Q, Q + 1]),
        parity=np.array([1.0, -1.0, -1.0, 1.0]), onsite=U * (nu @ nd),
        ops={"cu": cu, "cd": cd}, bond=bond,
        bonds=lambda L: [(i, i + 1, float(t), 0) for i in range(L - 1)],
        target=lambda n: (n // 2, n // 2), fermionic=True)


def chain(J=1.0):
    return lambda L: [(i, i + 1, float(J), 0) for i in range(L - 1)]


def j1j2(J1, J2):
    return lambda L: sorted([(i, i + 1, float(J1), 0) for i in range(L - 1)]
                            + [(i, i + 2, float(J2), 1) for i in range(L - 2)])


def ladder(j_leg=1.0, j_rung=1.0):
    """Two legs, sites numbered rung by rung (site = 2x + y); rungs group 0, legs 1."""
    def f(L):
        W = L // 2
        b = [(2 * x, 2 * x + 1, float(j_rung), 0) for x in range(W)]
        b += [(2 * x + y, 2 * x + 2 + y, float(j_leg), 1) for x in range(W - 1) for y in range(2)]
        return sorted(b)
    return f


# ---------------------------------------------------------------------------
# Block-sparse operators
# ---------------------------------------------------------------------------


@dataclass
class Basis:
    q: np.ndarray            # sector q, strictly increasing
    dim: np.ndarray          # sector sizes


@dataclass
class Op:
    delta: int
    blocks: dict             # (row sector, col sector) -> dense block

    def transpose(self):
        return Op(-self.delta, {(c, r): b.T.copy() for (r, c), b in self.blocks.items()})

    def scaled(self, rows=None, cols=None):
        """Multiply block (r, c) by rows[r] * cols[c] (per-sector scalars)."""
        out = {}
        for (r, c), b in self.blocks.items():
            f = (1.0 if rows is None else rows[r]) * (1.0 if cols is None else cols[c])
            out[(r, c)] = f * b
        return Op(self.delta, out)


def add_into(acc, op, c=1.0):
    for k, b in op.blocks.items():
        if k in acc:
            acc[k] = acc[k] + c * b
        else:
            acc[k] = c * b


@dataclass
class Block:
    labels: list
    basis: Basis
    H: dict                  # group -> {(r, r): block}
    ops: dict = field(default_factory=dict)   # (label, name) -> Op
    # how a truncated block came about: the grown product it was cut from and,
    # per kept sector k, (product sector, kept eigenvectors dim x kept)
    origin: object = None
    product: object = None   # for a grown block: its Product structure


def site_block(model, label, Q):
    q = model.qsite(Q)
    order = np.argsort(q, kind="stable")
    qs = q[order]
    if len(np.unique(qs)) != len(qs):
        raise ValueError("one-site states must have distinct quantum numbers")
    basis = Basis(qs.astype(np.int64), np.ones(len(qs), dtype=np.int64))
    H = {-1: {(i, i): model.onsite[order][:, order][i:i + 1, i:i + 1].copy()
              for i in range(len(qs)) if model.onsite[order[i], order[i]] != 0.0}}
    ops = {}
    for name, o in model.ops.items():
        oo = o[np.ix_(order, order)]
        blocks = {(i, j): oo[i:i + 1, j:j + 1].copy() for i in range(len(qs)) for j in range(len(qs))
                  if oo[i, j] != 0.0}
        deltas = {int(qs[i] - qs[j]) for (i, j) in blocks}
        ops[(label, name)] = Op(deltas.pop() if deltas else 0, blocks)
    return Block([label], basis, H, ops)


def sector_parity(basis, Q, fermionic):
    if not fermionic:
        return np.ones(len(basis.q))
    n = basis.q % Q + basis.q // Q
    return np.where(n % 2 == 0, 1.0, -1.0)


def _add_kron(blk, o1, o2, Lb, nl, Rb, nr):
    """blk[o1:, o2:] += Lb (x) Rb (None: the identity of size nl or nr).

    Where one factor is a single entry (a one-state sector, as every sector
    of a one-site basis with distinct quantum numbers is) the product is the
    other factor scaled, written straight into blk (the same products, one
    per entry, as the Kronecker product)."""
    if (Rb is None and nr == 1) or (Rb is not None and Rb.shape == (1, 1)):
        r = 1.0 if Rb is None else Rb[0, 0]
        if Lb is None:
            i = np.arange(nl)
            blk[o1 + i, o2 + i] += r
        else:
            blk[o1:o1 + Lb.shape[0], o2:o2 + Lb.shape[1]] += Lb * r
        return
    if (Lb is None and nl == 1) or (Lb is not None and Lb.shape == (1, 1)):
        l = 1.0 if Lb is None else Lb[0, 0]
        if Rb is None:
            i = np.arange(nr)
            blk[o1 + i, o2 + i] += l
        else:
            blk[o1:o1 + Rb.shape[0], o2:o2 + Rb.shape[1]] += l * Rb
        return
    sub = np.kron(np.eye(nl) if Lb is None else Lb, np.eye(nr) if Rb is None else Rb)
    blk[o1:o1 + sub.shape[0], o2:o2 + sub.shape[1]] += sub


class Product:
    """The basis of L (x) R, reordered by q: per product sector, its runs
    (left sector, right sector, offset) in product order."""

    def __init__(self, left: Basis, right: Basis, left_major=True):
        self.left, self.right = left, right
        self.left_major = left_major
        runs = {}
        for a in range(len(left.q)):
            for b in range(len(right.q)):
                runs.setdefault(int(left.q[a] + right.q[b]), []).append((a, b))
        qs = sorted(runs)
        self.basis = Basis(np.array(qs, dtype=np.int64), np.zeros(len(qs), dtype=np.int64))
        self.runs = []
        for s, qq in enumerate(qs):
            # product order: left index major (left_major) -- runs of one
            # sector in left-sector order; each run is dim(a) * dim(b) states
            rr = sorted(runs[qq]) if left_major else sorted(runs[qq], key=lambda t: (t[1], t[0]))
            off = 0
            lst = []
            for (a, b) in rr:
                lst.append((a, b, off))
                off += int(left.dim[a] * right.dim[b])
            self.runs.append(lst)
            self.basis.dim[s] = off
        self.index = {qq: s for s, qq in enumerate(qs)}

    def kron(self, A, a):
        """(A (x) a) on the product basis; A on the left part, a on the right
        (None: identity).  Both Op, or None."""
        L, R = self.left, self.right
        dA = 0 if A is None else A.delta
        da = 0 if a is None else a.delta
        Ab = None if A is None else A.blocks
        ab = None if a is None else a.blocks
        out = {}
        for s_out, runs_out in enumerate(self.runs):
            q_in = int(self.basis.q[s_out]) - dA - da
            s_in = self.index.get(q_in)
            if s_in is None:
                continue
            blk = None
            for (a1, b1, o1) in runs_out:
                for (a2, b2, o2) in self.runs[s_in]:
                    if Ab is None:
                        if a1 != a2:
                            continue
                        Lb = None
                    else:
                        Lb = Ab.get((a1, a2))
                        if Lb is None:
                            continue
                    if ab is None:
                        if b1 != b2:
                            continue
                        Rb = None
                    else:
                        Rb = ab.get((b1, b2))
                        if Rb is None:
                            continue
                    if blk is None:
                        blk = np.zeros((int(self.basis.dim[s_out]), int(self.basis.dim[s_in])))
                    _add_kron(blk, o1, o2, Lb, int(L.dim[a1]), Rb, int(R.dim[b1]))
            if blk is not None and np.any(blk != 0.0):
                out[(s_out, s_in)] = blk
        return Op(dA + da, out)


def _op(block, label, name, transpose):
    o = block.ops[(label, name)]
    return o.transpose() if transpose else o


def _bond_terms(model, left, right, label_l, label_r, value, Q):
    """[(c, A, B)] of one bond between a left and a right part."""
    Fl = sector_parity(left.basis, Q, model.fermionic)
    out = []
    for (f, ln, lt, rn, rt, fm) in model.bond:
        A = _op(left, label_l, ln, lt)
        if fm == "OF":
            A = A.scaled(cols=Fl)
        elif fm == "FO":
            A = A.scaled(rows=Fl)
        out.append((value * f, A, _op(right, label_r, rn, rt)))
    return out


def grow_right(S, model, Q, bonds, keep):
    """S' = S (x) x (Fig. 2(a))."""
    x = max(S.labels) + 1
    site = site_block(model, x, Q)
    P = Product(S.basis, site.basis, left_major=True)
    H = {}
    for g, blocks in S.H.items():
        H.setdefault(g, {})
        add_into(H[g], P.kron(Op(0, blocks), None))
    for g, blocks in site.H.items():
        H.setdefault(g, {})
        add_into(H[g], P.kron(None, Op(0, blocks)))
    for (i, j, v, g) in bonds:
        if j == x and i in S.labels:
            H.setdefault(g, {})
            for (c, A, B) in _bond_terms(model, S, site, i, x, v, Q):
                add_into(H[g], P.kron(A, B), c)
    FS = Op(0, {(r, r): np.diag(np.full(int(S.basis.dim[r]), f))
                for r, f in enumerate(sector_parity(S.basis, Q, model.fermionic))})
    ops = {}
    for (lab, name), o in S.ops.items():
        if lab > x - keep:
            ops[(lab, name)] = P.kron(o, None)
    for (lab, name), o in site.ops.items():
        ops[(lab, name)] = P.kron(FS if model.fermionic else None, o)
    return Block(S.labels + [x], P.basis, H, ops, product=P)


def grow_left(E, model, Q, n, bonds, keep):
    """E' = y (x) E (Fig. 2(b)); labels are distances from the right end."""
    r = max(E.labels) + 1
    site = site_block(model, r, Q)
    P = Product(site.basis, E.basis, left_major=True)
    H = {}
    for g, blocks in site.H.items():
        H.setdefault(g, {})
        add_into(H[g], P.kron(Op(0, blocks), None))
    for g, blocks in E.H.items():
        H.setdefault(g, {})
        add_into(H[g], P.kron(None, Op(0, blocks)))
    py = n - 1 - r
    for (i, j, v, g) in bonds:
        if i == py and (n - 1 - j) in E.labels:
            H.setdefault(g, {})
            for (c, A, B) in _bond_terms(model, site, E, r, n - 1 - j, v, Q):
                add_into(H[g], P.kron(A, B), c)
    Fy = Op(0, {(k, k): np.full((1, 1), f)
                for k, f in enumerate(sector_parity(site.basis, Q, model.fermionic))})
    ops = {}
    for (lab, name), o in site.ops.items():
        ops[(lab, name)] = P.kron(o, None)
    for (lab, name), o in E.ops.items():
        if lab > r - keep:
            ops[(lab, name)] = P.kron(Fy if model.fermionic else None, o)
    return Block(E.labels + [r], P.basis, H, ops, product=P)


def _as_desc_op(op):
    return None if op is None else dict(delta=int(op.delta),
                                         blocks=[(r, c, b) for (r, c), b in sorted(op.blocks.items())])


def superblock(Sp, Ep, model, Q, n, bonds, q_target):
    """Superblock description (terms H_S'(x)I, I(x)H_E' per group, bonds across)."""
    terms = []
    for g in sorted(Sp.H):
        if Sp.H[g]:
            terms.append(dict(c=1.0, A=_as_desc_op(Op(0, Sp.H[g])), B=None, group=g))
    for g in sorted(Ep.H):
        if Ep.H[g]:
            terms.append(dict(c=1.0, A=None, B=_as_desc_op(Op(0, Ep.H[g])), group=g))
    for (i, j, v, g) in bonds:
        if i in Sp.labels and (n - 1 - j) in Ep.labels:
            for (c, A, B) in _bond_terms(model, Sp, Ep, i, n - 1 - j, v, Q):
                terms.append(dict(c=c, A=_as_desc_op(A), B=_as_desc_op(B), group=g))
    return dict(S=dict(q=Sp.basis.q, dim=Sp.basis.dim), E=dict(q=Ep.basis.q, dim=Ep.basis.dim),
                q_target=int(q_target), terms=terms)


def change_basis(ctx, block, tr, product=None):
    """Truncate a grown block with the kept eigenvectors (Eq. (4)), on the GPU."""
    import torch
    W = tr["W"]
    keep_secs = sorted(W)
    new_index = {s: k for k, s in enumerate(keep_secs)}
    basis = Basis(np.array([block.basis.q[s] for s in keep_secs], dtype=np.int64),
                  np.array([W[s].shape[1] for s in keep_secs], dtype=np.int64))
    # every operator block whose row and column sectors survive
    items = []
    for g, blocks in block.H.items():
        for (r, c), b in blocks.items():
            items.append((("H", g), (r, c), b))
    for key, op in block.ops.items():
        for (r, c), b in op.blocks.items():
            items.append((("O", key), (r, c), b))
    items = [it for it in items if it[1][0] in W and it[1][1] in W]
    Wflat, woff = [], {}
    off = 0
    for s in keep_secs:
        woff[s] = off
        Wflat.append(W[s].reshape(-1))
        off += W[s].size
    Oflat, tbl = [], []
    o_off = out_off = 0
    for (_, (r, c), b) in items:
        tbl.append(dict(o_off=o_off, rows=b.shape[0], cols=b.shape[1], wr_off=woff[r],
                        kr=W[r].shape[1], wc_off=woff[c], kc=W[c].shape[1], out_off=out_off))
        Oflat.append(b.reshape(-1))
        o_off += b.size
        out_off += W[r].shape[1] * W[c].shape[1]
    new = Block(list(block.labels), basis, {g: {} for g in block.H},
                {k: Op(op.delta, {}) for k, op in block.ops.items()},
                origin=(product, [(s, W[s]) for s in keep_secs]))
    if not items:
        return new
    dO = torch.tensor(np.concatenate(Oflat), dtype=torch.float64, device=DEVICE)
    dW = torch.tensor(np.concatenate(Wflat), dtype=torch.float64, device=DEVICE)
    out = torch.empty(out_off, dtype=torch.float64, device=DEVICE)
    ctx.transform_blocks(tbl, dO, dW, out)
    res = out.cpu().numpy()
    for (kind, (r, c), _), t in zip(items, tbl):
        blk = res[t["out_off"]:t["out_off"] + t["kr"] * t["kc"]].reshape(t["kr"], t["kc"])
        key = (new_index[r], new_index[c])
        if kind[0] == "H":
            new.H[kind[1]][key] = blk.copy()
        else:
            new.ops[kind[1]].blocks[key] = blk.copy()
    return new


# ---------------------------------------------------------------------------
# Wave-function transformation between finite-sweep steps (the paper's
# conclusions, after White 1996): the previous ground state, written in the
# next superblock's basis, starts the next Lanczos run.  Each piece is
# Wr^T (slice of Psi) Wc, so the whole map is one dmrg_transform_blocks call.
# ---------------------------------------------------------------------------


def _pairs(sb):
    dS, dE = sb._dims
    return {(int(i), int(j)): (int(o), int(dS[i]), int(dE[j]))
            for i, j, o in zip(sb.s_sec, sb.e_sec, sb.offsets)}


def _runs_of(product, sector):
    return product.runs[sector]


def wf_left_to_right(ctx, old_sb, psi_old, PS_old, PE_old, W_L, left_new, right_old, new_sb,
                     PS_new, PE_new):
    """psi at split p -> start vector at split p+1.

    W_L: the kept eigenvectors of S'(p) (sector -> a x k), left_new = S'(p)
    truncated; right_old = R_{L-p-1}, whose origin expands it into
    site_{p+1} (x) R_{L-p-2} = E'(p+1)."""
    import torch
    old = _pairs(old_sb)
    new = _pairs(new_sb)
    keep_L = {s: k for k, (s, _w) in enumerate(left_new.origin[1])}
    R_prod, R_kept = right_old.origin
    Wbuf, tbl = [], []
    woff = [0]

    def put(a):
        Wbuf.append(np.ascontiguousarray(a).reshape(-1))
        o = woff[0]
        woff[0] += a.size
        return o

    wl_off = {s: put(W_L[s]) for s in W_L}
    wr_off = {k: put(Wk.T) for k, (_s, Wk) in enumerate(R_kept)}   # dim_rho x dim_rho'
    for (i, j), (o_ij, a, b) in old.items():
        if i not in W_L:
            continue
        li = keep_L[i]
        k_i = W_L[i].shape[1]
        for (x, rho, coff) in _runs_of(PE_old, j):
            sec_p, Wr = R_kept[rho]              # E'(p+1) sector and its kept vectors
            dim_rho = Wr.shape[1]
            q_new_S = int(PS_new.left.q[li] + PS_new.right.q[x])
            sig = PS_new.index.get(q_new_S)
            if sig is None:
                continue
            roff = next(o for (aa, bb, o) in PS_new.runs[sig] if aa == li and bb == x)
            if (sig, sec_p) not in new:
                continue
            n_off, _na, nb = new[(sig, sec_p)]
            tbl.append(dict(o_off=o_ij + coff, rows=a, cols=dim_rho, o_ld=b, wr_off=wl_off[i],
                            kr=k_i, wc_off=wr_off[rho], kc=Wr.shape[0],
                            out_off=n_off + roff * nb, out_ld=nb))
    out = torch.zeros(new_sb.D, dtype=torch.float64, device=DEVICE)
    if tbl:
        dW = torch.tensor(np.concatenate(Wbuf), dtype=torch.float64, device=DEVICE)
        ctx.transform_blocks(tbl, psi_old, dW, out)
    return out


def wf_right_to_left(ctx, old_sb, psi_old, PS_old, PE_old, W_E, right_new, left_old, new_sb,
                     PS_new, PE_new):
    """psi at split p -> start vector at split p-1 (the mirror image)."""
    import torch
    old = _pairs(old_sb)
    new = _pairs(new_sb)
    keep_E = {s: k for k, (s, _w) in enumerate(right_new.origin[1])}
    L_prod, L_kept = left_old.origin
    Wbuf, tbl = [], []
    woff = [0]

    def put(a):
        Wbuf.append(np.ascontiguousarray(a).reshape(-1))
        o = woff[0]
        woff[0] += a.size
        return o

    we_off = {s: put(W_E[s]) for s in W_E}
    wl_off = {k: put(Wk.T) for k, (_s, Wk) in enumerate(L_kept)}   # dim_a x dim_a'
    for (i, j), (o_ij, a, b) in old.items():
        if j not in W_E:
            continue
        rj = keep_E[j]
        k_j = W_E[j].shape[1]
        for (lam, x, roff) in _runs_of(PS_old, i):
            sec_p, Wl = L_kept[lam]               # S'(p-1) sector and its kept vectors
            dim_a = Wl.shape[1]
            q_new_E = int(PE_new.left.q[x] + PE_new.right.q[rj])
            tau = PE_new.index.get(q_new_E)
            if tau is None:
                continue
            coff = next(o for (aa, bb, o) in PE_new.runs[tau] if aa == x and bb == rj)
            if (sec_p, tau) not in new:
                continue
            n_off, _na, nb = new[(sec_p, tau)]
            tbl.append(dict(o_off=o_ij + roff * b, rows=dim_a, cols=b, o_ld=b, wr_off=wl_off[lam],
                            kr=Wl.shape[0], wc_off=we_off[j], kc=k_j,
                            out_off=n_off + coff, out_ld=nb))
    out = torch.zeros(new_sb.D, dtype=torch.float64, device=DEVICE)
    if tbl:
        dW = torch.tensor(np.concatenate(Wbuf), dtype=torch.float64, device=DEVICE)
        ctx.transform_blocks(tbl, psi_old, dW, out)
    return out


# ---------------------------------------------------------------------------
# Reflection symmetry in the infinite phase (the paper's conclusions: a factor
# of 2 in that phase).  When the n-site system is its own mirror image, the
# environment block of size h is the system block of size h read from the
# other end: same basis, same matrices, labels now distances from the right
# end.  Only S' is diagonalised and truncated.  Spin models only: for
# fermions the mirrored Jordan-Wigner strings would need a parity dressing.
# ---------------------------------------------------------------------------


def mirror_symmetric(model, n):
    b = {(i, j, v, g) for (i, j, v, g) in model.bonds(n)}
    m = {(n - 1 - j, n - 1 - i, v, g) for (i, j, v, g) in b}
    return b == m


def mirrored(block, model=None, Q=None):
    """The right block equal to a left block read from the other end.

    Its basis is the left block's read in reverse site order; for fermions
    each occupation configuration also takes the sign of reordering its
    creation operators from left-to-right to right-to-left site order,
    (-1)^(sum over site pairs i < j of n_i n_j).  With that basis every
    operator the right block carries (in its own Jordan-Wigner order, sites
    left to right) has the left block's matrix -- the block Hamiltonian and
    the site operators of mirrored sites alike -- so the matrices are shared
    for spins and fermions.  The origin is re-expressed in the site (x) block
    product order of a grown right block, so the wave-function
    transformation can expand it; for fermions the row of block state a and
    site state x takes the sign (-1)^(N_a n_x) that the reordering sign of a
    grown block adds to that of its block part."""
    origin = None
    if block.origin is not None and block.origin[0] is not None:
        Pl, kept = block.origin          # Pl = Product(left block, site)
        Pr = Product(Pl.right, Pl.left, left_major=True)   # site (x) block
        fermionic = model is not None and model.fermionic
        if fermionic:
            par_a = sector_parity(Pl.left, Q, True)          # (-1)^N_a per block sector
            n_x = Pl.right.q % Q + Pl.right.q // Q          # particles per site state
        new_kept = []
        for (sec, W) in kept:
            q = int(Pl.basis.q[sec])
            sec_r = Pr.index[q]
            rows = np.empty(W.shape[0], dtype=np.int64)
            sign = np.ones(W.shape[0])
            where = {(a, b): o for (a, b, o) in Pl.runs[sec]}
            for (x, a, o_r) in Pr.runs[sec_r]:
                o_l = where[(a, x)]
                n_run = int(Pl.left.dim[a] * Pl.right.dim[x])
                rows[o_r:o_r + n_run] = np.arange(o_l, o_l + n_run)
                if fermionic and n_x[x] % 2 == 1:
                    sign[o_r:o_r + n_run] = par_a[a]
            new_kept.append((sec_r, sign[:, None] * W[rows, :]))
        origin = (Pr, new_kept)
    return Block(list(block.labels), block.basis, block.H, dict(block.ops), origin=origin)


# ---------------------------------------------------------------------------
# Local density of states (Eq. (5)) by the continued-fraction method: c_i on
# the ground state through the library's sector-changing operator, the
# Lanczos recursion of H in the sector with one electron less from c_i|psi>,
# and the continued fraction on the host.
# ---------------------------------------------------------------------------


def ldos(ctx, Sp, Ep, model, n, q_target, psi, site, spin, omega, eta, nsteps=100,
         prec="fp64"):
    """N_site(omega) for spin 0 (up) / 1 (down) of the superblock's ground
    state psi; ``site`` is a label of S' (its newest site is max(Sp.labels))."""
    from .superblock import Superblock, ldos as host_ldos
    if not model.fermionic:
        raise ValueError("the local density of states needs a fermion model")
    name = "cu" if spin == 0 else "cd"
    if (site, name) not in Sp.ops:
        raise ValueError("site %r carries no operators in S'" % (site,))
    c_op = Sp.ops[(site, name)]               # c with its string inside S'
    q_out = q_target + c_op.delta
    op_desc = dict(S=dict(q=Sp.basis.q, dim=Sp.basis.dim), E=dict(q=Ep.basis.q, dim=Ep.basis.dim),
                   q_target=int(q_out), terms=[dict(c=1.0, A=_as_desc_op(c_op), B=None, group=0)])
    C_sb = Superblock(op_desc, prec="fp64", ctx=ctx, q_in=q_target)
    phi = C_sb.hpsi(psi)
    H_desc = superblock(Sp, Ep, model, _Q_of(Sp, Ep, model, n), n, model.bonds(n), q_out)
    H_sb = Superblock(H_desc, prec=prec, ctx=ctx)
    a, b, nrm = H_sb.lanczos_tridiag(phi, nsteps)
    C_sb.close()
    H_sb.close()
    return host_ldos(a, b, nrm * nrm, e0_of(ctx, Sp, Ep, model, n, q_target, psi, prec), omega,
                     eta)


def _Q_of(Sp, Ep, model, n):
    """The base of the effective quantum number the run used (Q = L + 1)."""
    return n + 1


def e0_of(ctx, Sp, Ep, model, n, q_target, psi, prec):
    """<psi|H|psi> of a normalised ground state (the E0 of Eq. (5))."""
    import torch

    from .superblock import Superblock
    desc = superblock(Sp, Ep, model, _Q_of(Sp, Ep, model, n), n, model.bonds(n), q_target)
    sb = Superblock(desc, prec="fp64", ctx=ctx)
    e0 = float(torch.dot(psi, sb.hpsi(psi)) / torch.dot(psi, psi))
    sb.close()
    return e0


def run(model, L, m, sweeps, init, ctx=None, prec="fp64", tol=1e-10, max_iter=2000,
        no_split=True, keep_range=None, on_step=None, wavefunction=True, reflect=False,
        on_solve=None, on_carry=None, checkpoint=None, resume=None, stop_after=None):
    """Infinite phase to L sites, then ``sweeps`` finite sweeps (Secs. 1, 3.1).

    ``init(D, step)`` gives the Lanczos start vector of each infinite-phase
    step (numpy); finite-sweep steps start from the previous ground state
    carried to the new basis when ``wavefunction`` is set (else ``init``).
    ``on_carry(info)``, if given, sees every carried vector with what made
    it (direction, old and new superblock bases, old ground state, the kept
    vectors used, the blocks involved).

    ``checkpoint`` (a path prefix): after every step the block stacks, the
    step records and the run's position go to ``<prefix>.blocks.npz`` and
    that step's superblock with its ground state to
    ``<prefix>.superblock.npz`` (see ``checkpoint.py``).  ``resume`` (a
    prefix written so) continues such a run with the same model, L, m and
    sweeps from the step after the saved one; its first step starts from
    ``init`` (the previous ground state is not kept).  ``stop_after=k``
    returns after k steps of this call (to end a run early on purpose).
    Returns a list of per-step records (those before a resume included).
    """
    import torch

    from .superblock import Context, Superblock
    if ctx is None:
        ctx = Context(0)
    Q = L + 1
    if keep_range is None:
        keep_range = max(j - i for (i, j, _v, _g) in model.bonds(L))
    left = {1: site_block(model, 0, Q)}
    right = {1: site_block(model, 0, Q)}
    log = []
    step = [0]
    prev = {}

    def solve(Sp, Ep, n, sides, phase, p, start=None, on=None):
        bonds = model.bonds(n)
        nu, nd = model.target(n)
        desc = superblock(Sp, Ep, model, Q, n, bonds, nu + Q * nd)
        sb = Superblock(desc, prec=prec, ctx=ctx)
        psi0 = start(sb) if start is not None else None
        if psi0 is None or float(torch.linalg.vector_norm(psi0)) == 0.0:
            psi0 = torch.tensor(init(sb.D, step[0]), dtype=torch.float64, device=DEVICE)
        r = sb.lanczos(psi0, max_iter=max_iter, tol=tol)
        rec = dict(phase=phase, n=n, p=p, energy=r["energy"], iters=r["iters"],
                   resid=r["resid"], D=sb.D, dimS=int(np.sum(Sp.basis.dim)),
                   dimE=int(np.sum(Ep.basis.dim)), step=step[0])
        out, trs = {}, {}
        for side in sides:
            tr = sb.rho_truncate(r["psi"], side, m, no_split=no_split)
            rec["eps%d" % side] = tr["eps"]
            rec["straddle%d" % side] = tr["straddle"]
            blk = Sp if side == 0 else Ep
            out[side] = change_basis(ctx, blk, tr, product=blk.product)
            trs[side] = tr
        if on is not None:
            on(rec, desc, r)
        elif on_step is not None:
            on_step(rec, desc, r)
        if on_solve is not None:
            on_solve(Sp, Ep, n, desc, r)
        log.append(rec)
        sb.close()
        step[0] += 1
        prev.clear()
        prev.update(sb=sb, psi=r["psi"], Sp=Sp, Ep=Ep, p=p, sides=sides, trs=trs, out=out,
                    phase=phase)
        return out

    # the whole run as one schedule: the infinite phase by size, then the
    # sweeps' (position, side) steps
    path = ([(p, 0) for p in range(L // 2, L - 1)] + [(p, 1) for p in range(L - 2, 1, -1)]
            + [(p, 0) for p in range(2, L // 2 + 1)])
    schedule = [("infinite", n, 0) for n in range(4, L + 1, 2)]
    schedule += [("finite", p, side) for _ in range(sweeps) for (p, side) in path]
    first = 0
    if resume is not None:
        from .checkpoint import load_blocks
        stacks, state = load_blocks(f"{resume}.blocks.npz")
        if (state["L"], state["m"], state["sweeps"], state["model"]) != (L, m, sweeps, model.name):
            raise ValueError(f"{resume}: checkpoint of another run ({state})")
        left, right = stacks["left"], stacks["right"]
        log[:] = state["log"]
        step[0] = state["step"]
        first = state["done"]

    def save(done, desc, psi):
        from .checkpoint import save_blocks, save_superblock
        save_superblock(f"{checkpoint}.superblock.npz", desc, psi.cpu().numpy())
        save_blocks(f"{checkpoint}.blocks.npz", {"left": left, "right": right},
                    state=dict(L=L, m=m, sweeps=sweeps, model=model.name, done=done, step=step[0],
                               log=log))

    last = {}

    def keep_last(rec, desc, r):
        last.update(desc=desc, psi=r["psi"])
        if on_step is not None:
            on_step(rec, desc, r)

    bonds = model.bonds(L)
    for i in range(first, len(schedule)):
        kind, a, side = schedule[i]
        if kind == "infinite":
            n = a
            h = n // 2
            nb = model.bonds(n)
            Sp = grow_right(left[h - 1], model, Q, nb, keep_range)
            Ep = grow_left(right[h - 1], model, Q, n, nb, keep_range)
            if reflect and mirror_symmetric(model, n):
                out = solve(Sp, Ep, n, (0,), "infinite", h, on=keep_last)
                left[h], right[h] = out[0], mirrored(out[0], model, Q)
            else:
                out = solve(Sp, Ep, n, (0, 1), "infinite", h, on=keep_last)
                left[h], right[h] = out[0], out[1]
        else:
            p = a
            Sp = grow_right(left[p - 1], model, Q, bonds, keep_range)
            Ep = grow_left(right[L - p - 1], model, Q, L, bonds, keep_range)
            start = None
            if wavefunction and prev:
                pv = dict(prev)
                same = pv["p"] == p and (pv["phase"] == "finite" or p == L // 2)
                if same:
                    start = lambda sb, pv=pv: pv["psi"] if sb.D == pv["sb"].D else None
                elif pv["p"] + 1 == p and 0 in pv["sides"]:
                    def start(sb, pv=pv, Sp=Sp, Ep=Ep, other=right[L - pv["p"] - 1]):
                        v = wf_left_to_right(ctx, pv["sb"], pv["psi"], pv["Sp"].product,
                                             pv["Ep"].product, pv["trs"][0]["W"], pv["out"][0],
                                             other, sb, Sp.product, Ep.product)
                        if on_carry is not None:
                            on_carry(dict(direction="left_to_right", p_old=pv["p"], p=p,
                                          old=(pv["Sp"].basis, pv["Ep"].basis), new=(Sp.basis, Ep.basis),
                                          psi_old=pv["psi"], W=pv["trs"][0]["W"], truncated=pv["out"][0],
                                          other=other, carried=v))
                        return v
                elif pv["p"] - 1 == p and 1 in pv["sides"]:
                    def start(sb, pv=pv, Sp=Sp, Ep=Ep, other=left[pv["p"] - 1]):
                        v = wf_right_to_left(ctx, pv["sb"], pv["psi"], pv["Sp"].product,
                                             pv["Ep"].product, pv["trs"][1]["W"], pv["out"][1],
                                             other, sb, Sp.product, Ep.product)
                        if on_carry is not None:
                            on_carry(dict(direction="right_to_left", p_old=pv["p"], p=p,
                                          old=(pv["Sp"].basis, pv["Ep"].basis), new=(Sp.basis, Ep.basis),
                                          psi_old=pv["psi"], W=pv["trs"][1]["W"], truncated=pv["out"][1],
                                          other=other, carried=v))
                        return v
            out = solve(Sp, Ep, L, (side,), "finite", p, start=start, on=keep_last)
            if side == 0:
                left[p] = out[0]
            else:
                right[L - p] = out[1]
        if checkpoint is not None:
            save(i + 1, last["desc"], last["psi"])
        if stop_after is not None and i + 1 - first >= stop_after:
            break
    return log
