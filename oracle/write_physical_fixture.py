"""Writes the centre superblock of an oracle DMRG run as a fixture file.

Test and benchmark infrastructure: it runs the oracle's infinite-phase DMRG
(Secs. 1 and 3.1; Hubbard chain, open boundaries, half filling) to L sites
with m kept states and stores the last superblock -- the one at the centre
split of the L-site chain, built from the truncated blocks of the run -- in
the superblock fixture layout that the library's checkpoint module reads
(numeric arrays plus one JSON header; no pickled objects).  The superblock
is physical: its sector sizes, operator blocks and coefficients are those
of the model after the run's truncations, not synthetic stand-ins.

    python -m oracle.write_physical_fixture --L 64 --U 4 --m 512 \
        --out workloads/data/hubbard_L64_U4_m512_physical.npz

The file's JSON header records the model, sizes, seed, the run's energies
and its wall time.  The writer here is independent of the library's own
(the two share no code); a CPU test reads the file with the library's
reader and checks it against the oracle.
"""
import argparse
import json
import os
import time

import numpy as np

from oracle import dmrg as OD
from oracle import models as M
from workloads import init_vector

FORMAT = 1


def _blocks(arrays, key, items):
    arrays[key + "_rc"] = np.array([(r, c) for (r, c, _) in items], dtype=np.int64).reshape(-1, 2)
    arrays[key + "_shape"] = np.array([b.shape for (_, _, b) in items], dtype=np.int64).reshape(-1, 2)
    arrays[key + "_data"] = (np.concatenate([np.asarray(b, dtype=np.float64).ravel() for (_, _, b) in items])
                             if items else np.zeros(0))


def write_fixture(path, desc, meta):
    arrays = {}
    terms = []
    for k, t in enumerate(desc["terms"]):
        rec = dict(c=float(t["c"]), group=int(t["group"]))
        for side in ("A", "B"):
            op = t[side]
            rec[side] = None if op is None else int(op["delta"])
            if op is not None:
                _blocks(arrays, f"t{k}_{side}", op["blocks"])
        terms.append(rec)
    for side in ("S", "E"):
        arrays[side + "_q"] = np.asarray(desc[side]["q"], dtype=np.int64)
        arrays[side + "_dim"] = np.asarray(desc[side]["dim"], dtype=np.int64)
    head = dict(format=FORMAT, kind="superblock", q_target=int(desc["q_target"]), terms=terms, meta=meta)
    arrays["header"] = np.array(json.dumps(head))
    tmp = path + ".tmp"
    with open(tmp, "wb") as f:
        np.savez_compressed(f, **arrays)
    os.replace(tmp, path)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--L", type=int, default=64)
    ap.add_argument("--U", type=float, default=4.0)
    ap.add_argument("--m", type=int, default=512)
    ap.add_argument("--tol", type=float, default=1e-9)
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    t0 = time.time()
    last = {}

    def on_superblock(phase, n, p, desc):
        last.update(desc=desc, n=n)
        print(f"[fixture] step n={n} D_S={int(np.sum(desc['S']['dim']))} ({time.time() - t0:.0f} s)", flush=True)

    log = OD.run(M.hubbard_model(args.U), args.L, args.m, 0, lambda D, step: init_vector(D, step),
                 tol=args.tol, on_superblock=on_superblock)
    assert last["n"] == args.L
    meta = dict(model="hubbard", L=args.L, U=args.U, t=1.0, m=args.m, filling="half",
                source="oracle infinite-phase DMRG, centre superblock of the last step",
                init="workloads.init_vector(D, step)", tol=args.tol,
                energies=[float(r["energy"]) for r in log], seconds=round(time.time() - t0, 1))
    write_fixture(args.out, last["desc"], meta)
    print(f"[fixture] wrote {args.out} ({os.path.getsize(args.out) / 2**20:.1f} MiB), "
          f"E0(L={args.L}) = {log[-1]['energy']:.12f}", flush=True)


if __name__ == "__main__":
    main()
