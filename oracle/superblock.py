"""The superblock product y = H psi (oracle; test infrastructure).

A superblock is described by plain data (no code is shared with the HIP
path; only the description format is common):

``S``, ``E``   bases of the grown system S' and environment E': dicts with
               ``q`` (effective quantum numbers of the sectors, strictly
               increasing) and ``dim`` (states per sector) -- the
               quantumNumbers/partition pair of Sec. 3.2.
``q_target``   the targeted effective quantum number (Sec. 3.3: only the
               symmetry blocks with the targeted numbers are diagonalised).
``terms``      H = sum_k c_k A_k (x) B_k.  Each term is a dict with ``c``,
               ``A`` (an operator on S' or None for the identity) and ``B``
               (an operator on E' or None).  An operator is a dict with
               ``delta`` (q(row) - q(col), the same for all of its blocks,
               Sec. 3.2: quantum numbers add) and ``blocks``, a list of
               (row sector, column sector, dense FP64 block).

The wave function psi (Eq. (1)) lives in the target sector only: the pairs
(i, j) of S' and E' sectors with q_S[i] + q_E[j] = q_target, ordered by i,
each stored as a row-major dim_S[i] x dim_E[j] matrix Psi_ij (rows: states
of S', columns: states of E'), one after the other.

Three evaluations of the same product are given:

* ``hpsi_kron``   the explicit Kronecker matrix H = sum c_k kron(A_k, B_k)
                  on the full product space (Sec. 3.3: C_{a1 b1; a2 b2} =
                  A_{a1 a2} B_{b1 b2}), restricted to the target sector.
* ``hpsi_dense``  (A (x) B) psi = A Psi B^T on the full dense Psi.
* ``hpsi_blocks`` per symmetry block, Y_q += c_k A_k[q <- q'] Psi_q' B_k^T
                  (Sec. 3.3: blocking the Hamiltonian by effective symmetry).
"""
from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------------------
# Layout
# ---------------------------------------------------------------------------

def offsets(dims):
    """Sector start offsets (the partition vector of Sec. 3.2)."""
    return np.concatenate([[0], np.cumsum(np.asarray(dims, dtype=np.int64))])


def target_pairs(sb):
    """Target pairs [(i, j, offset)] ordered by S' sector, and the total size D."""
    qS = np.asarray(sb["S"]["q"], dtype=np.int64)
    qE = np.asarray(sb["E"]["q"], dtype=np.int64)
    dS = np.asarray(sb["S"]["dim"], dtype=np.int64)
    dE = np.asarray(sb["E"]["dim"], dtype=np.int64)
    pairs = []
    off = 0
    for i in range(len(qS)):
        for j in range(len(qE)):
            if qS[i] + qE[j] == sb["q_target"]:
                pairs.append((i, j, off))
                off += int(dS[i] * dE[j])
    return pairs, off


def target_indices(sb):
    """Positions of the packed psi entries in the full (N_S * N_E) product space."""
    oS = offsets(sb["S"]["dim"])
    oE = offsets(sb["E"]["dim"])
    NE = int(oE[-1])
    pairs, D = target_pairs(sb)
    idx = np.empty(D, dtype=np.int64)
    for (i, j, off) in pairs:
        a = int(sb["S"]["dim"][i])
        b = int(sb["E"]["dim"][j])
        rows = oS[i] + np.arange(a)
        cols = oE[j] + np.arange(b)
        idx[off:off + a * b] = (rows[:, None] * NE + cols[None, :]).reshape(-1)
    return idx


def full_operator(op, basis):
    """Dense N x N matrix of a block operator (None -> identity)."""
    o = offsets(basis["dim"])
    N = int(o[-1])
    if op is None:
        return np.eye(N)
    M = np.zeros((N, N))
    for (r, c, blk) in op["blocks"]:
        M[o[r]:o[r + 1], o[c]:o[c + 1]] += blk
    return M


# ---------------------------------------------------------------------------
# y = H psi
# ---------------------------------------------------------------------------

def kron_matrix(sb):
    """The explicit superblock matrix sum_k c_k kron(A_k, B_k), target rows/cols."""
    idx = target_indices(sb)
    H = None
    for t in sb["terms"]:
        A = full_operator(t["A"], sb["S"])
        B = full_operator(t["B"], sb["E"])
        K = t["c"] * np.kron(A, B)
        H = K if H is None else H + K
    return H[np.ix_(idx, idx)]


def hpsi_kron(sb, psi):
    """y = H psi with H formed explicitly as a Kronecker sum (small cases)."""
    return kron_matrix(sb) @ psi


def unpack(sb, psi):
    """Packed target-sector psi -> full dense Psi (N_S x N_E), zero elsewhere."""
    NS = int(np.sum(sb["S"]["dim"]))
    NE = int(np.sum(sb["E"]["dim"]))
    full = np.zeros(NS * NE)
    full[target_indices(sb)] = psi
    return full.reshape(NS, NE)


def pack(sb, Psi):
    """Full dense Psi -> packed target-sector vector."""
    return Psi.reshape(-1)[target_indices(sb)]


def hpsi_dense(sb, psi):
    """y = sum_k c_k A_k Psi B_k^T on the dense product space, then the target part."""
    Psi = unpack(sb, psi)
    Y = np.zeros_like(Psi)
    for t in sb["terms"]:
        A = full_operator(t["A"], sb["S"])
        B = full_operator(t["B"], sb["E"])
        Y += t["c"] * (A @ Psi @ B.T)
    return pack(sb, Y)


def _block_map(op):
    """row sector -> (column sector, block); None for the identity."""
    if op is None:
        return None
    m = {}
    for (r, c, blk) in op["blocks"]:
        if r in m:
            raise ValueError("two blocks in one row sector")
        m[r] = (c, blk)
    return m


def _apply_side(bmap, sec):
    """(source sector, block or None for identity) for output sector ``sec``."""
    if bmap is None:
        return sec, None
    if sec not in bmap:
        return None, None
    return bmap[sec]


def hpsi_blocks(sb, psi, coeffs=None):
    """y = H psi evaluated per symmetry block: Y_(i,j) += c A[i<-i'] Psi_(i',j') B[j<-j']^T."""
    pairs, D = target_pairs(sb)
    where = {(i, j): off for (i, j, off) in pairs}
    dS = sb["S"]["dim"]
    dE = sb["E"]["dim"]
    y = np.zeros(D)
    terms = sb["terms"]
    cs = [t["c"] for t in terms] if coeffs is None else list(coeffs)
    maps = [(_block_map(t["A"]), _block_map(t["B"])) for t in terms]
    for (i, j, off) in pairs:
        a, b = int(dS[i]), int(dE[j])
        Y = y[off:off + a * b].reshape(a, b)
        for c, (mA, mB) in zip(cs, maps):
            i2, Ablk = _apply_side(mA, i)
            j2, Bblk = _apply_side(mB, j)
            if i2 is None or j2 is None or (i2, j2) not in where:
                continue
            o2 = where[(i2, j2)]
            X = psi[o2:o2 + int(dS[i2]) * int(dE[j2])].reshape(int(dS[i2]), int(dE[j2]))
            T = X if Ablk is None else Ablk @ X
            T = T if Bblk is None else T @ Bblk.T
            Y += c * T
    return y


# ---------------------------------------------------------------------------
# The adjoint: grad_psi = H^T g and grad_c_k = <g, (A_k (x) B_k) psi>
# ---------------------------------------------------------------------------

def hpsi_adjoint_dense(sb, psi, g):
    """(H^T g, [<g, (A_k (x) B_k) psi>]_k) from the dense definition."""
    Psi = unpack(sb, psi)
    G = unpack(sb, g)
    GP = np.zeros_like(Psi)
    gc = []
    for t in sb["terms"]:
        A = full_operator(t["A"], sb["S"])
        B = full_operator(t["B"], sb["E"])
        GP += t["c"] * (A.T @ G @ B)
        gc.append(float(np.sum(G * pack_mask(sb, A @ Psi @ B.T))))
    return pack(sb, GP), np.array(gc)


def pack_mask(sb, M):
    """Zero a dense N_S x N_E matrix outside the target sector."""
    out = np.zeros_like(M)
    idx = target_indices(sb)
    out.reshape(-1)[idx] = M.reshape(-1)[idx]
    return out


def hpsi_adjoint_blocks(sb, psi, g):
    """H^T g and the per-term inner products, evaluated per symmetry block."""
    pairs, D = target_pairs(sb)
    where = {(i, j): off for (i, j, off) in pairs}
    dS = sb["S"]["dim"]
    dE = sb["E"]["dim"]
    gp = np.zeros(D)
    gc = np.zeros(len(sb["terms"]))
    for k, t in enumerate(sb["terms"]):
        mA, mB = _block_map(t["A"]), _block_map(t["B"])
        for (i, j, off) in pairs:
            i2, Ablk = _apply_side(mA, i)
            j2, Bblk = _apply_side(mB, j)
            if i2 is None or j2 is None or (i2, j2) not in where:
                continue
            a, b = int(dS[i]), int(dE[j])
            a2, b2 = int(dS[i2]), int(dE[j2])
            o2 = where[(i2, j2)]
            G = g[off:off + a * b].reshape(a, b)
            X = psi[o2:o2 + a2 * b2].reshape(a2, b2)
            T = X if Ablk is None else Ablk @ X
            T = T if Bblk is None else T @ Bblk.T
            gc[k] += float(np.sum(G * T))
            U = G if Ablk is None else Ablk.T @ G
            U = U if Bblk is None else U @ Bblk
            gp[o2:o2 + a2 * b2] += t["c"] * U.reshape(-1)
    return gp, gc


# ---------------------------------------------------------------------------
# Checks of a description (Sec. 3.2: quantum numbers add under the product)
# ---------------------------------------------------------------------------

def check_quantum_numbers(sb):
    """Raise if a block breaks q(row) - q(col) = delta or a term is not q-neutral."""
    for t in sb["terms"]:
        dA = 0 if t["A"] is None else t["A"]["delta"]
        dB = 0 if t["B"] is None else t["B"]["delta"]
        if dA + dB != 0:
            raise ValueError("term changes the total quantum number")
        for side, basis in (("A", sb["S"]), ("B", sb["E"])):
            op = t[side]
            if op is None:
                continue
            for (r, c, blk) in op["blocks"]:
                if basis["q"][r] - basis["q"][c] != op["delta"]:
                    raise ValueError("block breaks the operator's q shift")
                if blk.shape != (basis["dim"][r], basis["dim"][c]):
                    raise ValueError("block shape does not match the sectors")


# ---------------------------------------------------------------------------
# Single entries, for sampled checks at sizes where the full product is slow
# ---------------------------------------------------------------------------

def hpsi_element(sb, psi, i, j, m, n, absolute=False):
    """Entry (m, n) of block (i, j) of H psi from the definition,
    sum_k c_k sum_{a', b'} A_k[m, a'] Psi'[a', b'] B_k[n, b'].

    With ``absolute`` every factor is replaced by its absolute value, which
    gives the scale (|H| |psi|) that rounding errors are measured against.
    """
    pairs, _ = target_pairs(sb)
    where = {(p[0], p[1]): p[2] for p in pairs}
    dS, dE = sb["S"]["dim"], sb["E"]["dim"]
    f = np.abs if absolute else (lambda x: x)
    total = 0.0
    for t in sb["terms"]:
        i2, Ablk = _apply_side(_block_map(t["A"]), i)
        j2, Bblk = _apply_side(_block_map(t["B"]), j)
        if i2 is None or j2 is None or (i2, j2) not in where:
            continue
        o2 = where[(i2, j2)]
        X = f(psi[o2:o2 + int(dS[i2]) * int(dE[j2])].reshape(int(dS[i2]), int(dE[j2])))
        a = np.zeros(int(dS[i2]))
        if Ablk is None:
            a[m] = 1.0
        else:
            a = f(Ablk[m, :])
        b = np.zeros(int(dE[j2]))
        if Bblk is None:
            b[n] = 1.0
        else:
            b = f(Bblk[n, :])
        total += f(t["c"]) * float(a @ X @ b)
    return total


def abs_description(sb):
    """The description with every coefficient and block entry replaced by its
    absolute value (so that hpsi of |psi| gives |H| |psi|)."""
    def op(o):
        if o is None:
            return None
        return dict(delta=o["delta"], blocks=[(r, c, np.abs(b)) for (r, c, b) in o["blocks"]])
    return dict(S=sb["S"], E=sb["E"], q_target=sb["q_target"],
                terms=[dict(c=abs(t["c"]), A=op(t["A"]), B=op(t["B"]), group=t.get("group", 0))
                       for t in sb["terms"]])
