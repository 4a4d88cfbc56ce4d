"""Entry-by-entry rounding bounds for the GPU product (test helper).

For one entry y_i = sum_p x_p of n_i nonzero products x_p, any summation
order in floating point with unit roundoff u leaves |fl(y_i) - y_i| <=
(n_i - 1) u sum_p |x_p| (to first order; adding an exact zero rounds
nothing).  sum_p |x_p| is (|H| |psi|)_i, the product with every coefficient,
block entry and vector entry replaced by its absolute value, and n_i is the
same product on the 0/1 pattern of the blocks with a vector of ones.

Per product the reduced-precision paths also round their operands before
the contraction: the block entry to FP32, the coefficient to FP32 and their
product, psi to FP32, the gather scale to FP32 and their product, then the
product of the two; seven roundings in all (``OPERAND_ROUNDINGS``, with
three more of slack).  The BF16 split writes each FP32 operand x as
hi + lo + r with hi = bf16(x), lo = bf16(x - hi) (8 significant bits each,
round to nearest), so |r| <= 2^-16 |x| and |lo| <= 2^-8 (1 + 2^-8) |x|;
dropping lo*lo and the two remainders leaves at most
((1 + 2^-8)^2 + 2 (1 + 2^-16) + 2^-16) 2^-16 |x_a x_b| per product, and each
product is accumulated as three FP32 additions.
"""
import numpy as np

from oracle import superblock as OS

U = {"fp64": 2.0 ** -53, "fp64_plain": 2.0 ** -53, "fp32": 2.0 ** -24, "bf16x3": 2.0 ** -24}
OPERAND_ROUNDINGS = 10
BF16_SPLIT = ((1 + 2.0 ** -8) ** 2 + 2 * (1 + 2.0 ** -16) + 2.0 ** -16) * 2.0 ** -16
ADDS_PER_PRODUCT = {"fp64": 1, "fp64_plain": 1, "fp32": 1, "bf16x3": 3}


def pattern_description(sb):
    """The description with coefficient 1 and every block replaced by its
    0/1 nonzero pattern: its product with a vector of ones counts, entry by
    entry, the nonzero products the true product sums."""
    def op(o):
        if o is None:
            return None
        return dict(delta=o["delta"],
                    blocks=[(r, c, (b != 0.0).astype(float)) for (r, c, b) in o["blocks"]])
    return dict(S=sb["S"], E=sb["E"], q_target=sb["q_target"],
                terms=[dict(c=1.0, A=op(t["A"]), B=op(t["B"]), group=t.get("group", 0))
                       for t in sb["terms"]])


def relative_bound(prec, n):
    """Bound on |error| / (|H||psi|)_i for an entry that sums n nonzero products."""
    u = U[prec]
    split = BF16_SPLIT if prec == "bf16x3" else 0.0
    return split + (ADDS_PER_PRODUCT[prec] * n + OPERAND_ROUNDINGS) * u


def product_bound(sb, psi, prec):
    """(scale s_i = (|H||psi|)_i, bound_i) for every entry of H psi."""
    _, D = OS.target_pairs(sb)
    s = OS.hpsi_blocks(OS.abs_description(sb), np.abs(psi))
    n = OS.hpsi_blocks(pattern_description(sb), np.ones(D))
    return s, relative_bound(prec, n) * s * (1 + 1e-6)


def adjoint_bound(sb, psi, g, prec):
    """Bounds for H^T g (entry by entry) and for each term's <g, A_k (x) B_k psi>.

    Each term's inner product sums FP64 products of g with that term's tile
    values (each within its own product bound) over the D entries, so
    |error_k| <= sum_i |g_i| bound_ik + D 2^-53 sum_i |g_i| s_ik."""
    _, D = OS.target_pairs(sb)
    ab = OS.abs_description(sb)
    pat = pattern_description(sb)
    s_t = OS.hpsi_adjoint_blocks(ab, np.abs(psi), np.abs(g))[0]
    n_t = OS.hpsi_adjoint_blocks(pat, np.ones(D), np.ones(D))[0]
    gp_bound = relative_bound(prec, n_t) * s_t * (1 + 1e-6)
    gc_bound = np.zeros(len(sb["terms"]))
    for k in range(len(sb["terms"])):
        e = np.zeros(len(sb["terms"]))
        e[k] = 1.0
        s_k = OS.hpsi_blocks(ab, np.abs(psi), coeffs=e)
        n_k = OS.hpsi_blocks(pat, np.ones(D), coeffs=e)
        per = relative_bound(prec, n_k) * s_k
        gc_bound[k] = (float(np.dot(np.abs(g), per))
                       + D * 2.0 ** -53 * float(np.dot(np.abs(g), s_k))) * (1 + 1e-6)
    return s_t, gp_bound, gc_bound
