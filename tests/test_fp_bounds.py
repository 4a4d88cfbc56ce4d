"""CPU checks of the rounding bounds the GPU parity tests use.

The product is evaluated here in FP32 and in the BF16 hi/lo split with
numpy, block by block, rounding the operands as the reduced-precision
paths do; every entry must stay inside fp_bounds' bound, and the bound must
not be vacuous (a dropped term, a sign flip or an index off by one breaks it).
"""
import numpy as np
import pytest

from oracle import superblock as OS
from workloads import seeded_vector, workload_superblock

import fp_bounds as FB

from test_oracle_superblock import SMALL
from workloads import make_superblock


def _bf16(x):
    """Round float32 values to bfloat16 (round to nearest even), kept as float32."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def _mm(prec, A, X):
    if prec == "fp32":
        return A @ X
    ah, xh = _bf16(A), _bf16(X)
    al, xl = _bf16(A - ah), _bf16(X - xh)
    return (ah @ xh + ah @ xl) + al @ xh


def _emulated(sb, psi, prec):
    """H psi per symmetry block with FP32 operands (the BF16 split on the
    contraction when asked); elementwise (identity) terms in FP64."""
    pairs, D = OS.target_pairs(sb)
    where = {(i, j): off for (i, j, off) in pairs}
    dS, dE = sb["S"]["dim"], sb["E"]["dim"]
    y = np.zeros(D)
    p32 = psi.astype(np.float32)
    maps = [(OS._block_map(t["A"]), OS._block_map(t["B"])) for t in sb["terms"]]
    for (i, j, off) in pairs:
        a, b = int(dS[i]), int(dE[j])
        for t, (mA, mB) in zip(sb["terms"], maps):
            i2, Ablk = OS._apply_side(mA, i)
            j2, Bblk = OS._apply_side(mB, j)
            if i2 is None or j2 is None or (i2, j2) not in where:
                continue
            o2 = where[(i2, j2)]
            shape = (int(dS[i2]), int(dE[j2]))
            if Ablk is None and Bblk is None:
                y[off:off + a * b] += t["c"] * psi[o2:o2 + a * b]
                continue
            X = p32[o2:o2 + shape[0] * shape[1]].reshape(shape)
            c32 = np.float32(t["c"])
            T = _mm(prec, c32 * Ablk.astype(np.float32), X) if Ablk is not None else c32 * X
            if Bblk is not None:
                T = _mm(prec, T, Bblk.astype(np.float32).T)
            y[off:off + a * b] += T.astype(np.float64).reshape(-1)
    return y


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("k", range(len(SMALL)))
def test_emulated_reduced_precision_within_bound(k, prec):
    sb = make_superblock(seed=3, **SMALL[k])
    _, D = OS.target_pairs(sb)
    psi = seeded_vector(D, 9)
    ref = OS.hpsi_blocks(sb, psi)
    s, bound = FB.product_bound(sb, psi, prec)
    err = np.abs(_emulated(sb, psi, prec) - ref)
    assert np.all(err <= bound), (prec, float(np.max(err / np.maximum(bound, 1e-300))))


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_emulated_reduced_precision_within_bound_workload(prec):
    sb = workload_superblock("hubbard_L64_U4_m512", m=64, seed=1)
    _, D = OS.target_pairs(sb)
    psi = seeded_vector(D, 10)
    ref = OS.hpsi_blocks(sb, psi)
    s, bound = FB.product_bound(sb, psi, prec)
    err = np.abs(_emulated(sb, psi, prec) - ref)
    assert np.all(err <= bound)


def test_bound_catches_planted_mistakes():
    """Entry-wise bounds are tight enough to fail a dropped term, a flipped
    coefficient sign or an index off by one (planted in a copy of the
    oracle's input, on the CPU)."""
    sb = workload_superblock("j1j2_L64_m256", m=48, seed=1)
    _, D = OS.target_pairs(sb)
    psi = seeded_vector(D, 11)
    ref = OS.hpsi_blocks(sb, psi)
    _, bound = FB.product_bound(sb, psi, "bf16x3")
    k = next(k for k, t in enumerate(sb["terms"]) if t["A"] is not None and t["B"] is not None)
    c = np.array([t["c"] for t in sb["terms"]])
    dropped = c.copy()
    dropped[k] = 0.0
    flipped = c.copy()
    flipped[k] = -c[k]
    for cc in (dropped, flipped):
        assert np.any(np.abs(OS.hpsi_blocks(sb, psi, coeffs=cc) - ref) > bound)
    # an index off by one: the rows of every block of one operator rolled
    bad = dict(sb, terms=[dict(t) for t in sb["terms"]])
    A = sb["terms"][k]["A"]
    bad["terms"][k] = dict(sb["terms"][k], A=dict(A, blocks=[
        (r, cc, np.roll(blk, 1, axis=0)) for (r, cc, blk) in A["blocks"]]))
    assert np.any(np.abs(OS.hpsi_blocks(bad, psi) - ref) > bound)


def test_pattern_counts_are_products():
    """The pattern product counts the nonzero products of each entry: it is
    at least 1 wherever the absolute product is positive, and summing it
    over entries gives the total count from the blocks' nonzeros directly."""
    sb = make_superblock(seed=3, **SMALL[0])
    pairs, D = OS.target_pairs(sb)
    s = OS.hpsi_blocks(OS.abs_description(sb), np.ones(D))
    n = OS.hpsi_blocks(FB.pattern_description(sb), np.ones(D))
    assert np.all(n[s > 0] >= 1) and np.all(n[s == 0] == 0)
    where = {(i, j) for (i, j, _o) in pairs}
    dS, dE = sb["S"]["dim"], sb["E"]["dim"]
    total = 0
    for t in sb["terms"]:
        mA, mB = OS._block_map(t["A"]), OS._block_map(t["B"])
        for (i, j, _o) in pairs:
            i2, Ablk = OS._apply_side(mA, i)
            j2, Bblk = OS._apply_side(mB, j)
            if i2 is None or j2 is None or (i2, j2) not in where:
                continue
            ra = np.ones(int(dS[i])) if Ablk is None else np.count_nonzero(Ablk, axis=1)
            rb = np.ones(int(dE[j])) if Bblk is None else np.count_nonzero(Bblk, axis=1)
            total += int(np.sum(np.outer(ra, rb)))
    assert int(round(np.sum(n))) == total
