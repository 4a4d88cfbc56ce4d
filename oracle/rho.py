"""Reduced density matrices and truncation (oracle; test infrastructure).

Eq. (2): (rho_S)_{a,a'} = sum_b psi*_{a',b} psi_{a,b}, i.e. rho_S = Psi Psi^dag
(Psi Psi^T for real psi); Eq. (3): rho_E = Psi^T Psi*.  Both commute with the
effective quantum number (Sec. 3.2: the DMRG transformation preserves it), so
they are diagonalised sector by sector.  The eigenvectors are ordered by
decreasing eigenvalue, the first m are kept -- all of them when m is at least
the dimension (Sec. 1) -- and the truncation error is the sum of the
discarded eigenvalues (Sec. 1).  The kept eigenvectors W change the basis of
block operators as O -> W^T O W (Eq. (4), reading (w^S)^{-1} as W^T, which is
what a rectangular, column-orthonormal W admits; Sec. 3.3: W^dag W = 1).

The paper gives no rule for equal eigenvalues at the cut.  Reading used on
both sides of every comparison:

1. eigenvalues below ``floor`` (1e-13) count as 0;
2. sort by eigenvalue, largest first;
3. neighbours in that order whose eigenvalues differ by at most
   ``rel_tie`` (1e-6) times the larger belong to one cluster (all zeros form
   one cluster);
4. inside a cluster, order by effective q ascending, then by position in
   the sector's own decreasing order;
5. ``no_split`` keeps the whole cluster the m-th state falls in, unless it
   is the zero cluster; otherwise exactly m states are kept.
"""
from __future__ import annotations

import numpy as np

from .superblock import target_pairs

FLOOR = 1e-13
REL_TIE = 1e-6


def density_blocks(sb, psi, side):
    """{sector: rho block} for every sector of S' (side 0) or E' (side 1)."""
    pairs, _ = target_pairs(sb)
    basis = sb["S"] if side == 0 else sb["E"]
    dS, dE = sb["S"]["dim"], sb["E"]["dim"]
    out = {s: np.zeros((int(basis["dim"][s]),) * 2) for s in range(len(basis["dim"]))}
    for (i, j, off) in pairs:
        a, b = int(dS[i]), int(dE[j])
        P = psi[off:off + a * b].reshape(a, b)
        if side == 0:
            out[i] += P @ P.T
        else:
            out[j] += P.T @ P
    return out


def spectrum_order(entries, floor=FLOOR, rel_tie=REL_TIE):
    """Order [(lam, q, idx, sector)] by the tie-break rule; returns (order, cluster ids)."""
    lam = np.array([max(e[0], 0.0) if e[0] >= floor else 0.0 for e in entries])
    first = sorted(range(len(entries)),
                   key=lambda k: (-lam[k], entries[k][1], entries[k][2]))
    clusters = []
    cid = 0
    for pos, k in enumerate(first):
        if pos > 0:
            p = first[pos - 1]
            a, b = lam[p], lam[k]
            tied = (a == 0.0 and b == 0.0) or abs(a - b) <= rel_tie * max(a, b)
            if not tied:
                cid += 1
        clusters.append(cid)
    order = []
    pos = 0
    while pos < len(first):
        end = pos
        while end < len(first) and clusters[end] == clusters[pos]:
            end += 1
        block = sorted(first[pos:end], key=lambda k: (entries[k][1], entries[k][2]))
        order += block
        pos = end
    return order, clusters, lam


def truncate(sb, psi, side, m, no_split=False):
    """Density-matrix truncation of S' (side 0) or E' (side 1) to m states.

    Returns dict(eps, kept, lam (kept, in order), lam_sec (sector of each
    kept value), W {sector: dim x kept matrix}, straddle (bool), all_lam).
    """
    basis = sb["S"] if side == 0 else sb["E"]
    blocks = density_blocks(sb, psi, side)
    entries = []
    vecs = {}
    for s in range(len(basis["dim"])):
        w, U = np.linalg.eigh(blocks[s])
        w, U = w[::-1], U[:, ::-1]
        vecs[s] = U
        for k in range(len(w)):
            entries.append((float(w[k]), int(basis["q"][s]), k, s))
    order, clusters, lam = spectrum_order(entries)
    n = len(entries)
    keep = n if m >= n else m
    straddle = False
    if keep < n:
        # cluster of the last kept entry vs the first discarded one
        c_last = clusters[keep - 1]
        c_next = clusters[keep]
        straddle = c_last == c_next and lam[order[keep]] > 0.0
        if no_split and straddle:
            while keep < n and clusters[keep] == c_last:
                keep += 1
    kept = order[:keep]
    disc = order[keep:]
    eps = float(sum(lam[k] for k in disc))
    per_sec = {}
    for k in kept:
        per_sec.setdefault(entries[k][3], []).append(entries[k][2])
    W = {s: vecs[s][:, sorted(idx)] for s, idx in per_sec.items()}
    return dict(eps=eps, kept=keep,
                lam=np.array([entries[k][0] for k in kept]),
                lam_sec=np.array([entries[k][3] for k in kept]),
                W=W, straddle=straddle,
                all_lam=np.array([e[0] for e in entries]))


def transform_block(O, Wr, Wc):
    """One block of the basis change, Eq. (4) with (w)^-1 read as W^T:
    O_new = Wr^T O Wc, Wr / Wc the kept eigenvectors of the row / column sector."""
    return Wr.T @ O @ Wc
