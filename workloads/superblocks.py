"""Synthetic superblocks with the shapes of the five model workloads.

A superblock is the product of a grown system S' = S (x) x and a grown
environment E' = y (x) E at the centre of an L-site chain.  Here S and E
are synthetic truncated blocks: their m states are spread over
symmetry sectors by a discretised Gaussian in the conserved numbers
(N_up for spin chains; (N_up, N_down) for Hubbard) centred at half filling
and capped by the sector's full size, assigned one state at a time to the
sector with the largest weight / (states so far + 1).  The products with the
new sites are reordered by effective q (stable), which gives the sector
tables of S' and E'.

Operators (all float64, row-major dense blocks per sector pair):

* block Hamiltonians H_S', H_E': per sector Q diag(e) Q^T, Q a seeded
  random orthogonal matrix, e_i = w sqrt(i / a) + kappa |n - n_c|^2
  (a sparse low end and a penalty away from half filling, so the
  superblock ground state is gapped like a physical one);
* operators on the newest sites x and y: I_S (x) o and o (x) I_E for the
  one-site matrices o of the model -- at most one nonzero per row;
* operators on the older boundary sites (ladder and J1-J2 only): seeded
  random dense blocks with the operator's q shift, N(0,1)/sqrt(dim) scaled,
  transposes paired so that H stays symmetric.

The term lists follow the bonds that cross the S'|E' cut:
nearest-neighbour chains have one bond (x, y); the two-leg ladder (sites
numbered rung by rung, cut after an even site) and the J1-J2 chain have
(x, y), (s, y) and (x, e) with s the last site of S and e the first of E.
"""
from __future__ import annotations

import json
import os
from math import comb

import numpy as np

# name -> workload parameters
WORKLOADS = {
    "heisenberg_L16_m32": dict(model="spin", L=16, m=32, bonds="chain", sigma=1.4),
    "heisenberg_L100_m256": dict(model="spin", L=100, m=256, bonds="chain", sigma=1.35),
    "hubbard_L64_U4_m512": dict(model="hubbard", L=64, m=512, bonds="chain", sigma=1.15,
                                U=4.0, t=1.0),
    "ladder_2x32_m1024": dict(model="spin", L=64, m=1024, bonds="ladder", sigma=1.9),
    "j1j2_L64_m256": dict(model="spin", L=64, m=256, bonds="j1j2", sigma=1.35),
}


# --- one-site tables --------------------------------------------------------

def _spin_site():
    # states (down, up); q = N_up
    sz = np.diag([-0.5, 0.5])
    spl = np.zeros((2, 2))
    spl[1, 0] = 1.0                 # S^+ |down> = |up>
    return dict(d=2, nup=np.array([0, 1]), ndn=np.array([0, 0]), Sz=sz, Sp=spl)


def _hubbard_site():
    # states (e, up, down, updown); |updown> = c^dag_up c^dag_down |e>
    c_up = np.zeros((4, 4))
    c_dn = np.zeros((4, 4))
    c_up[0, 1] = 1.0
    c_up[2, 3] = 1.0
    c_dn[0, 2] = 1.0
    c_dn[1, 3] = -1.0
    F = np.diag([1.0, -1.0, -1.0, 1.0])
    return dict(d=4, nup=np.array([0, 1, 0, 1]), ndn=np.array([0, 0, 1, 1]),
                c_up=c_up, c_dn=c_dn, F=F)


# --- sector recipes ---------------------------------------------------------

def block_sectors(model, nsites, m, sigma):
    """[(n_up, n_down, dim)] of a synthetic truncated block of nsites sites."""
    c = nsites / 2.0
    cands = []
    if model == "spin":
        for nu in range(nsites + 1):
            cands.append((nu, 0, comb(nsites, nu), np.exp(-(nu - c) ** 2 / (2 * sigma ** 2))))
    else:
        for nu in range(nsites + 1):
            for nd in range(nsites + 1):
                w = np.exp(-((nu - c) ** 2 + (nd - c) ** 2) / (2 * sigma ** 2))
                cands.append((nu, nd, comb(nsites, nu) * comb(nsites, nd), w))
    total = min(m, sum(x[2] for x in cands))
    dims = [0] * len(cands)
    for _ in range(total):
        best, bestv = -1, -1.0
        for k, (_nu, _nd, cap, w) in enumerate(cands):
            if dims[k] < cap:
                v = w / (dims[k] + 1)
                if v > bestv:
                    best, bestv = k, v
        dims[best] += 1
    return [(cands[k][0], cands[k][1], dims[k]) for k in range(len(cands)) if dims[k] > 0]


def _expand(secs, Q):
    """Per-state (q, n_up, n_down) of a block listed sector by sector (q ascending)."""
    rows = sorted(secs, key=lambda s: s[0] + Q * s[1])
    q, nu, nd = [], [], []
    for (a, b, dim) in rows:
        q += [a + Q * b] * dim
        nu += [a] * dim
        nd += [b] * dim
    return np.array(q, dtype=np.int64), np.array(nu), np.array(nd)


def _product(qL, qR):
    """Stable reorder of the product states (l, r) -> index l*nR + r by q."""
    q = (qL[:, None] + qR[None, :]).reshape(-1)
    perm = np.argsort(q, kind="stable")
    pos = np.empty_like(perm)
    pos[perm] = np.arange(len(perm))
    return q[perm], pos


def _sector_table(q_sorted):
    u, cnt = np.unique(q_sorted, return_counts=True)
    start = np.concatenate([[0], np.cumsum(cnt)])
    return u.astype(np.int64), cnt.astype(np.int64), start


# --- operators --------------------------------------------------------------

def _to_blocks(rows, cols, vals, start, qsec):
    """Sparse (row, col, value) in a sorted basis -> {'delta', 'blocks'} dense blocks."""
    sec_of = np.searchsorted(start, np.arange(start[-1]), side="right") - 1
    blocks = {}
    deltas = set()
    for r, c, v in zip(rows, cols, vals):
        sr, sc = int(sec_of[r]), int(sec_of[c])
        key = (sr, sc)
        if key not in blocks:
            blocks[key] = np.zeros((start[sr + 1] - start[sr], start[sc + 1] - start[sc]))
            deltas.add(int(qsec[sr] - qsec[sc]))
        blocks[key][r - start[sr], c - start[sc]] += v
    assert len(deltas) <= 1
    return dict(delta=deltas.pop() if deltas else 0,
                blocks=[(k[0], k[1], b) for k, b in sorted(blocks.items())])


def _site_op_on_product(o, nblock, d, pos, side):
    """I_block (x) o (side 'right': site on the right) or o (x) I_block, as triplets."""
    rows, cols, vals = [], [], []
    nz = np.argwhere(o != 0.0)
    for (xr, xc) in nz:
        v = o[xr, xc]
        for s in range(nblock):
            if side == "right":
                rows.append(pos[s * d + xr])
                cols.append(pos[s * d + xc])
            else:
                rows.append(pos[xr * nblock + s])
                cols.append(pos[xc * nblock + s])
            vals.append(v)
    return rows, cols, vals


def _orthogonal(a, rng):
    X = rng.standard_normal((a, a))
    Qm, R = np.linalg.qr(X)
    return Qm * np.sign(np.diag(R))[None, :]


def _block_hamiltonian(qsec, cnt, nsites, Q, model, rng, w=6.0, kappa=0.5):
    blocks = []
    c = nsites / 2.0
    for s, (qq, a) in enumerate(zip(qsec, cnt)):
        nu, nd = int(qq % Q), int(qq // Q)
        pen = kappa * ((nu - c) ** 2 + ((nd - c) ** 2 if model == "hubbard" else 0.0))
        e = w * np.sqrt(np.arange(a) / max(a, 1)) + pen
        Qm = _orthogonal(int(a), rng)
        H = (Qm * e[None, :]) @ Qm.T
        blocks.append((s, s, 0.5 * (H + H.T)))
    return dict(delta=0, blocks=blocks)


def _dense_op(qsec, cnt, delta, rng, scale=0.5):
    """Seeded dense blocks mapping sector q - delta -> q."""
    where = {int(q): k for k, q in enumerate(qsec)}
    blocks = []
    for r, qq in enumerate(qsec):
        c = where.get(int(qq) - delta)
        if c is None:
            continue
        B = rng.standard_normal((int(cnt[r]), int(cnt[c]))) * scale / np.sqrt(max(cnt[c], 1))
        if delta == 0:
            B = 0.5 * (B + B.T)
        blocks.append((r, c, B))
    return dict(delta=delta, blocks=blocks)


def _transpose(op):
    return dict(delta=-op["delta"], blocks=[(c, r, b.T.copy()) for (r, c, b) in op["blocks"]])


# --- superblocks ------------------------------------------------------------

def make_superblock(model, L, m, bonds="chain", sigma=1.5, seed=0, U=4.0, t=1.0,
                    j1=1.0, j2=None, j_leg=1.0, j_rung=1.0):
    """A synthetic centre-cut superblock of an L-site system keeping m states."""
    rng = np.random.default_rng([int(seed), 7])
    Q = L + 1 if model == "hubbard" else 1 << 20
    site = _spin_site() if model == "spin" else _hubbard_site()
    d = site["d"]
    qsite = site["nup"] + (Q * site["ndn"] if model == "hubbard" else 0)
    nS = L // 2 - 1
    nE = L - L // 2 - 1
    qS_states, _, _ = _expand(block_sectors(model, nS, m, sigma), Q)
    qE_states, _, _ = _expand(block_sectors(model, nE, m, sigma), Q)
    qSp, posS = _product(qS_states, qsite)          # S' = S (x) x
    qEp, posE = _product(qsite, qE_states)          # E' = y (x) E
    qsS, cS, stS = _sector_table(qSp)
    qsE, cE, stE = _sector_table(qEp)
    nS_states, nE_states = len(qS_states), len(qE_states)

    def right_site(o):   # operator on x inside S'
        return _to_blocks(*_site_op_on_product(o, nS_states, d, posS, "right"), stS, qsS)

    def left_site(o):    # operator on y inside E'
        return _to_blocks(*_site_op_on_product(o, nE_states, d, posE, "left"), stE, qsE)

    if model == "hubbard":
        nup, ndn = L // 2, L // 2
    else:
        nup, ndn = L // 2, 0
    q_target = nup + (Q * ndn if model == "hubbard" else 0)
    S = dict(q=qsS, dim=cS)
    E = dict(q=qsE, dim=cE)
    terms = []
    meta = dict(model=model, L=L, m=m, bonds=bonds, seed=seed)
    if model == "hubbard":
        terms.append(dict(c=1.0, A=_block_hamiltonian(qsS, cS, nS + 1, Q, model, rng), B=None, group=0))
        terms.append(dict(c=1.0, A=None, B=_block_hamiltonian(qsE, cE, nE + 1, Q, model, rng), group=0))
        F = site["F"]
        for s in ("c_up", "c_dn"):
            c = site[s]
            # t (c^dag_x F) (x) c_y  and  t (F c_x) (x) c^dag_y
            terms.append(dict(c=t, A=right_site(c.T @ F), B=left_site(c), group=1))
            terms.append(dict(c=t, A=right_site(F @ c), B=left_site(c.T), group=1))
        meta.update(U=U, t=t)
    else:
        groups = {"chain": 1, "ladder": 2, "j1j2": 2}[bonds]
        if bonds == "j1j2":
            if j2 is None:
                j2 = float(np.random.default_rng([int(seed), 11]).uniform(0.0, 0.5))
            couplings = [j1, j2]
        elif bonds == "ladder":
            couplings = [j_rung, j_leg]
        else:
            couplings = [j1]
        for g in range(groups):
            terms.append(dict(c=couplings[g], A=_block_hamiltonian(qsS, cS, nS + 1, Q, model, rng),
                              B=None, group=g))
            terms.append(dict(c=couplings[g], A=None,
                              B=_block_hamiltonian(qsE, cE, nE + 1, Q, model, rng), group=g))
        Sz, Sp = site["Sz"], site["Sp"]
        xz, xp = right_site(Sz), right_site(Sp)
        yz, yp = left_site(Sz), left_site(Sp)

        def spin_bond(c, Az, Ap, Bz, Bp, g):
            terms.append(dict(c=c, A=Az, B=Bz, group=g))
            terms.append(dict(c=0.5 * c, A=Ap, B=_transpose(Bp), group=g))
            terms.append(dict(c=0.5 * c, A=_transpose(Ap), B=Bp, group=g))

        if bonds == "chain":
            spin_bond(j1, xz, xp, yz, yp, 0)
        else:
            # (x, y): rung / J1; (s, y) and (x, e): leg / J2 (older sites are dense)
            g_xy, g_long = (0, 1)
            c_xy = couplings[0]
            c_long = couplings[1]
            sz_dense = _dense_op(qsS, cS, 0, rng)
            sp_dense = _dense_op(qsS, cS, 1, rng)
            ez_dense = _dense_op(qsE, cE, 0, rng)
            ep_dense = _dense_op(qsE, cE, 1, rng)
            spin_bond(c_xy, xz, xp, yz, yp, g_xy)
            spin_bond(c_long, sz_dense, sp_dense, yz, yp, g_long)
            spin_bond(c_long, xz, xp, ez_dense, ep_dense, g_long)
        meta.update(couplings=couplings)
    return dict(S=S, E=E, q_target=int(q_target), terms=terms, meta=meta)


# Stored superblocks (files under data/, written by oracle/write_physical_fixture.py
# from the oracle's own DMRG run): name -> file
FIXTURES = {
    "hubbard_L64_U4_m512_physical": "hubbard_L64_U4_m512_physical.npz",
}
DATA = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")


def fixture_superblock(name):
    """A stored superblock description (the layout of the fixture files:
    numeric arrays plus one JSON header, read without unpickling)."""
    with np.load(os.path.join(DATA, FIXTURES[name]), allow_pickle=False) as z:
        arrays = {k: z[k] for k in z.files}
    head = json.loads(str(arrays["header"]))
    terms = []
    for k, rec in enumerate(head["terms"]):
        t = dict(c=rec["c"], group=rec["group"])
        for side in ("A", "B"):
            if rec[side] is None:
                t[side] = None
                continue
            key = f"t{k}_{side}"
            blocks, off = [], 0
            data = arrays[key + "_data"]
            for (r, c), (mr, nc) in zip(arrays[key + "_rc"], arrays[key + "_shape"]):
                blocks.append((int(r), int(c), data[off:off + mr * nc].reshape(mr, nc)))
                off += int(mr) * int(nc)
            t[side] = dict(delta=rec[side], blocks=blocks)
        terms.append(t)
    return dict(S=dict(q=arrays["S_q"], dim=arrays["S_dim"]), E=dict(q=arrays["E_q"], dim=arrays["E_dim"]),
                q_target=head["q_target"], terms=terms, meta=head.get("meta", {}))


def workload_superblock(name, seed=0, m=None, L=None):
    """The superblock of a named workload: synthetic (optionally a reduced m
    or L), or a stored one (no size options)."""
    if name in FIXTURES:
        if m is not None or L is not None:
            raise ValueError(f"{name} is a stored superblock: no m or L")
        return fixture_superblock(name)
    p = dict(WORKLOADS[name])
    kw = dict(model=p["model"], L=p["L"] if L is None else L, m=p["m"] if m is None else m,
              bonds=p["bonds"], sigma=p["sigma"], seed=seed)
    if p["model"] == "hubbard":
        kw.update(U=p["U"], t=p["t"])
    return make_superblock(**kw)
