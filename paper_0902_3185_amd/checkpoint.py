"""Superblock fixtures and DMRG checkpoints as .npz files.

The finite algorithm keeps a copy of every block it grows on a last-in,
first-out stack and reads them back on the sweeps (Sec. 3.1, the infinite
loop's push of the system block); the paper keeps those stacks in memory
and names stacks on disk as future work (Sec. 5).  Here:

* ``save_superblock`` / ``load_superblock``: one superblock description --
  the sector tables of S' and E', the target sector, and per term its
  coefficient, group and the dense symmetry blocks of A_k and B_k (what
  dmrg_build_superblock takes) -- plus, optionally, a vector such as the
  ground state.  A loaded description builds the same superblock.
* ``save_blocks`` / ``load_blocks``: the driver's block stacks (per block
  its site labels, sector table, Hamiltonian blocks per coupling group,
  operator blocks and how it was cut from its grown product), the state a
  run resumes from.

Files are written with ``numpy.savez_compressed`` and read with
``numpy.load(allow_pickle=False)``: numeric arrays and one JSON text entry,
nothing that runs code when it is loaded.  Writes go to a temporary file in
the same folder and are renamed into place, so a run killed while writing
leaves the previous file whole.
"""
from __future__ import annotations

import json
import os

import numpy as np

FORMAT = 1


def _plain(o):
    """JSON form of the numpy scalars a record may hold."""
    if isinstance(o, np.generic):
        return o.item()
    raise TypeError(f"not JSON serialisable: {type(o).__name__}")


def _write(path, arrays):
    path = os.fspath(path)
    d = os.path.dirname(os.path.abspath(path))
    tmp = os.path.join(d, "." + os.path.basename(path) + ".tmp")
    with open(tmp, "wb") as f:
        np.savez_compressed(f, **arrays)
    os.replace(tmp, path)


def _read(path):
    with np.load(os.fspath(path), allow_pickle=False) as z:
        arrays = {k: z[k] for k in z.files}
    head = json.loads(str(arrays.pop("header")))
    if head.get("format") != FORMAT:
        raise ValueError(f"{path}: unknown checkpoint format {head.get('format')}")
    return head, arrays


def _put_blocks(arrays, key, items):
    """items: list of (row sector, col sector, 2-D array) -> three arrays."""
    rc = np.array([(r, c) for (r, c, _) in items], dtype=np.int64).reshape(-1, 2)
    shp = np.array([b.shape for (_, _, b) in items], dtype=np.int64).reshape(-1, 2)
    data = (np.concatenate([np.ascontiguousarray(b, dtype=np.float64).ravel() for (_, _, b) in items])
            if items else np.zeros(0))
    arrays[key + "_rc"] = rc
    arrays[key + "_shape"] = shp
    arrays[key + "_data"] = data


def _get_blocks(arrays, key):
    rc = arrays[key + "_rc"]
    shp = arrays[key + "_shape"]
    data = arrays[key + "_data"]
    out, off = [], 0
    for (r, c), (m, n) in zip(rc, shp):
        out.append((int(r), int(c), data[off:off + m * n].reshape(m, n).copy()))
        off += int(m) * int(n)
    if off != data.size:
        raise ValueError(f"{key}: block data does not match the block shapes")
    return out


def save_superblock(path, desc, psi=None):
    """Write a superblock description (and optionally a vector) to ``path``."""
    arrays = {}
    terms = []
    for k, t in enumerate(desc["terms"]):
        rec = dict(c=float(t["c"]), group=int(t.get("group", 0)))
        for side in ("A", "B"):
            op = t[side]
            if op is None:
                rec[side] = None
                continue
            rec[side] = int(op["delta"])
            _put_blocks(arrays, f"t{k}_{side}", list(op["blocks"]))
        terms.append(rec)
    for side in ("S", "E"):
        arrays[side + "_q"] = np.asarray(desc[side]["q"], dtype=np.int64)
        arrays[side + "_dim"] = np.asarray(desc[side]["dim"], dtype=np.int64)
    if psi is not None:
        arrays["psi"] = np.asarray(psi, dtype=np.float64)
    head = dict(format=FORMAT, kind="superblock", q_target=int(desc["q_target"]), terms=terms,
                meta=desc.get("meta", {}))
    arrays["header"] = np.array(json.dumps(head, default=_plain))
    _write(path, arrays)


def load_superblock(path):
    """(description, vector or None) from a file written by save_superblock."""
    head, arrays = _read(path)
    if head.get("kind") != "superblock":
        raise ValueError(f"{path}: not a superblock fixture")
    terms = []
    for k, rec in enumerate(head["terms"]):
        t = dict(c=rec["c"], group=rec["group"])
        for side in ("A", "B"):
            t[side] = (None if rec[side] is None
                       else dict(delta=rec[side], blocks=_get_blocks(arrays, f"t{k}_{side}")))
        terms.append(t)
    desc = dict(S=dict(q=arrays["S_q"], dim=arrays["S_dim"]), E=dict(q=arrays["E_q"], dim=arrays["E_dim"]),
                q_target=head["q_target"], terms=terms)
    if head.get("meta"):
        desc["meta"] = head["meta"]
    return desc, arrays.get("psi")


def save_blocks(path, stacks, state=None):
    """Write block stacks to ``path``.

    ``stacks`` maps a stack name to {position: Block} (the driver's ``left``
    and ``right``); ``state`` is any JSON-serialisable record of where the
    run stands.  Kept per block: labels, sectors, Hamiltonian blocks per
    group, operator blocks and, for a truncated block, how it was cut (the
    grown product's two bases and the kept vectors per product sector), which
    the carried start vectors need."""
    arrays = {}
    index = {}
    for name, stack in stacks.items():
        index[name] = {}
        for pos, blk in stack.items():
            key = f"{name}{int(pos)}"
            rec = dict(labels=[int(x) for x in blk.labels], H=[], ops=[])
            arrays[key + "_q"] = np.asarray(blk.basis.q, dtype=np.int64)
            arrays[key + "_dim"] = np.asarray(blk.basis.dim, dtype=np.int64)
            for gi, (g, blocks) in enumerate(sorted(blk.H.items())):
                rec["H"].append(int(g))
                _put_blocks(arrays, f"{key}_H{gi}", [(r, c, b) for (r, c), b in sorted(blocks.items())])
            for oi, ((lab, op_name), op) in enumerate(sorted(blk.ops.items())):
                rec["ops"].append([int(lab), str(op_name), int(op.delta)])
                _put_blocks(arrays, f"{key}_O{oi}", [(r, c, b) for (r, c), b in sorted(op.blocks.items())])
            if blk.origin is not None:
                # how the block was cut: the grown product (rebuilt from its
                # two bases) and the kept vectors per product sector
                P, kept = blk.origin
                for side, b in (("L", P.left), ("R", P.right)):
                    arrays[f"{key}_P{side}_q"] = np.asarray(b.q, dtype=np.int64)
                    arrays[f"{key}_P{side}_dim"] = np.asarray(b.dim, dtype=np.int64)
                rec["origin"] = dict(left_major=bool(P.left_major), sectors=[int(s) for (s, _w) in kept])
                _put_blocks(arrays, f"{key}_W", [(int(s), 0, w) for (s, w) in kept])
            index[name][str(int(pos))] = rec
    head = dict(format=FORMAT, kind="blocks", index=index, state=state)
    arrays["header"] = np.array(json.dumps(head, default=_plain))
    _write(path, arrays)


def load_blocks(path):
    """({name: {position: Block}}, state) from a file written by save_blocks."""
    from .driver import Basis, Block, Op, Product
    head, arrays = _read(path)
    if head.get("kind") != "blocks":
        raise ValueError(f"{path}: not a block-stack checkpoint")
    stacks = {}
    for name, entries in head["index"].items():
        stack = {}
        for pos, rec in entries.items():
            key = f"{name}{int(pos)}"
            basis = Basis(arrays[key + "_q"], arrays[key + "_dim"])
            H = {}
            for gi, g in enumerate(rec["H"]):
                H[g] = {(r, c): b for (r, c, b) in _get_blocks(arrays, f"{key}_H{gi}")}
            ops = {}
            for oi, (lab, op_name, delta) in enumerate(rec["ops"]):
                ops[(lab, op_name)] = Op(delta, {(r, c): b for (r, c, b) in _get_blocks(arrays, f"{key}_O{oi}")})
            origin = None
            if rec.get("origin"):
                P = Product(Basis(arrays[f"{key}_PL_q"], arrays[f"{key}_PL_dim"]),
                            Basis(arrays[f"{key}_PR_q"], arrays[f"{key}_PR_dim"]),
                            left_major=rec["origin"]["left_major"])
                origin = (P, [(s, w) for (s, _c, w) in _get_blocks(arrays, f"{key}_W")])
            stack[int(pos)] = Block(list(rec["labels"]), basis, H, ops, origin=origin)
        stacks[name] = stack
    return stacks, head.get("state")
