"""Pins of the oracle's superblock product, Lanczos and truncation (CPU only)."""
import numpy as np
import pytest

from oracle import dmrg as OD
from oracle import lanczos as OL
from oracle import models as M
from oracle import rho as OR
from oracle import superblock as OS
from workloads import make_superblock, seeded_vector

SMALL = [
    dict(model="spin", L=16, m=8, bonds="chain", sigma=1.4),
    dict(model="hubbard", L=10, m=12, bonds="chain", sigma=1.0),
    dict(model="spin", L=12, m=10, bonds="ladder", sigma=1.2),
    dict(model="spin", L=12, m=10, bonds="j1j2", sigma=1.2),
]


@pytest.fixture(params=range(len(SMALL)), ids=[s["model"] + "-" + s["bonds"] for s in SMALL])
def small_sb(request):
    sb = make_superblock(seed=3, **SMALL[request.param])
    OS.check_quantum_numbers(sb)
    return sb


def test_blocks_equal_kronecker(small_sb):
    _, D = OS.target_pairs(small_sb)
    psi = seeded_vector(D, 1)
    yk = OS.hpsi_kron(small_sb, psi)
    yd = OS.hpsi_dense(small_sb, psi)
    yb = OS.hpsi_blocks(small_sb, psi)
    scale = np.linalg.norm(yk)
    assert np.linalg.norm(yb - yk) <= 1e-13 * scale
    assert np.linalg.norm(yd - yk) <= 1e-13 * scale


def test_kronecker_single_term_by_hand():
    # one sector each side, A (x) B on a 2x3 product: y[a,b] = sum A[a,a'] B[b,b'] x[a',b']
    A = np.array([[1.0, 2.0], [3.0, 4.0]])
    B = np.array([[0.0, 1.0, 0.0], [1.0, 0.0, 2.0], [0.0, 5.0, 1.0]])
    sb = dict(S=dict(q=np.array([0]), dim=np.array([2])), E=dict(q=np.array([0]), dim=np.array([3])),
              q_target=0, terms=[dict(c=2.0, A=dict(delta=0, blocks=[(0, 0, A)]),
                                      B=dict(delta=0, blocks=[(0, 0, B)]))])
    x = np.arange(6.0)
    X = x.reshape(2, 3)
    want = np.zeros((2, 3))
    for a in range(2):
        for b in range(3):
            for a2 in range(2):
                for b2 in range(3):
                    want[a, b] += 2.0 * A[a, a2] * B[b, b2] * X[a2, b2]
    assert np.allclose(OS.hpsi_kron(sb, x), want.reshape(-1))
    assert np.allclose(OS.hpsi_blocks(sb, x), want.reshape(-1))


def test_hermitian_and_sector_closed(small_sb):
    _, D = OS.target_pairs(small_sb)
    x, y = seeded_vector(D, 2), seeded_vector(D, 3)
    lhs = np.dot(x, OS.hpsi_blocks(small_sb, y))
    rhs = np.dot(OS.hpsi_blocks(small_sb, x), y)
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)
    # a target-sector vector has no image outside the target sector
    NS, NE = int(np.sum(small_sb["S"]["dim"])), int(np.sum(small_sb["E"]["dim"]))
    full = np.zeros(NS * NE)
    idx = OS.target_indices(small_sb)
    full[idx] = x
    Y = np.zeros((NS, NE))
    X = full.reshape(NS, NE)
    for t in small_sb["terms"]:
        Y += t["c"] * OS.full_operator(t["A"], small_sb["S"]) @ X @ OS.full_operator(
            t["B"], small_sb["E"]).T
    mask = np.ones(NS * NE, bool)
    mask[idx] = False
    assert np.max(np.abs(Y.reshape(-1)[mask])) == 0.0


def test_adjoint(small_sb):
    _, D = OS.target_pairs(small_sb)
    psi, g = seeded_vector(D, 4), seeded_vector(D, 5)
    gp_b, gc_b = OS.hpsi_adjoint_blocks(small_sb, psi, g)
    gp_d, gc_d = OS.hpsi_adjoint_dense(small_sb, psi, g)
    assert np.allclose(gp_b, gp_d, atol=1e-12)
    assert np.allclose(gc_b, gc_d, atol=1e-12)
    # <g, H psi> = <H^T g, psi> and d<g, H(c) psi>/dc_k (H is linear in c)
    assert abs(np.dot(g, OS.hpsi_blocks(small_sb, psi)) - np.dot(gp_b, psi)) < 1e-11
    c0 = np.array([t["c"] for t in small_sb["terms"]])
    for k in range(len(c0)):
        cp, cm = c0.copy(), c0.copy()
        cp[k] += 0.5
        cm[k] -= 0.5
        fd = np.dot(g, OS.hpsi_blocks(small_sb, psi, cp)) - np.dot(g, OS.hpsi_blocks(small_sb, psi, cm))
        assert abs(fd - gc_b[k]) < 1e-11


def test_superblock_without_truncation_is_exact():
    # Hubbard n=6: S' and E' are 3-site blocks (64 states) kept whole -> ED
    L = 6
    model = M.hubbard_model(2.0)
    Q = L + 1
    bonds = model.bonds(L)
    S = OD.site_block(model, 0, Q)
    S = OD.grow_right(S, model, Q, bonds, 1)
    S = OD.grow_right(S, model, Q, bonds, 1)
    E = OD.site_block(model, 0, Q)
    E = OD.grow_left(E, model, Q, L, bonds, 1)
    E = OD.grow_left(E, model, Q, L, bonds, 1)
    terms = OD.superblock_terms(S, E, model, Q, L, bonds)
    sb = OD.describe(S, E, terms, 3 + Q * 3)
    Hk = OS.kron_matrix(sb)
    e0 = np.linalg.eigvalsh(Hk)[0]
    assert abs(e0 - M.hubbard_ed(L, bonds, 2.0)[0]) < 1e-11


def test_lanczos_matches_eigh():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((300, 300))
    H = X + X.T + np.diag(np.arange(300) * 0.1)
    w, V = np.linalg.eigh(H)
    E, psi, it, res = OL.lanczos_ground(lambda v: H @ v, seeded_vector(300, 0), tol=1e-11)
    assert abs(E - w[0]) < 1e-9
    assert abs(abs(np.dot(psi, V[:, 0])) - 1) < 1e-9
    assert res < 1e-9


def test_lanczos_breakdown_on_eigenvector():
    H = np.diag([1.0, 2.0, 3.0])
    E, psi, it, res = OL.lanczos_ground(lambda v: H @ v, np.array([0.0, 1.0, 0.0]))
    assert it == 1 and abs(E - 2.0) < 1e-15 and res < 1e-15


def test_lanczos_on_superblock(small_sb):
    _, D = OS.target_pairs(small_sb)
    w = np.linalg.eigvalsh(OS.kron_matrix(small_sb))
    E, psi, it, res = OL.lanczos_ground(lambda v: OS.hpsi_blocks(small_sb, v),
                                        seeded_vector(D, 9), tol=1e-10)
    assert abs(E - w[0]) < 1e-9


def _normalised_psi(sb, seed):
    _, D = OS.target_pairs(sb)
    v = seeded_vector(D, seed)
    return v / np.linalg.norm(v)


def test_density_matrix_properties(small_sb):
    psi = _normalised_psi(small_sb, 11)
    rS = OR.density_blocks(small_sb, psi, 0)
    rE = OR.density_blocks(small_sb, psi, 1)
    assert abs(sum(np.trace(b) for b in rS.values()) - 1) < 1e-13
    assert abs(sum(np.trace(b) for b in rE.values()) - 1) < 1e-13
    lS = np.sort(np.concatenate([np.linalg.eigvalsh(b) for b in rS.values()]))[::-1]
    lE = np.sort(np.concatenate([np.linalg.eigvalsh(b) for b in rE.values()]))[::-1]
    # Schmidt: the nonzero spectra agree, and equal the squared singular values
    pairs, _ = OS.target_pairs(small_sb)
    sv = []
    for (i, j, off) in pairs:
        a, b = int(small_sb["S"]["dim"][i]), int(small_sb["E"]["dim"][j])
        sv += list(np.linalg.svd(psi[off:off + a * b].reshape(a, b), compute_uv=False) ** 2)
    sv = np.sort(np.array(sv))[::-1]
    k = len(sv)
    assert np.allclose(lS[:k], sv, atol=1e-14)
    assert np.allclose(lE[:k], sv, atol=1e-14)
    assert np.all(np.abs(lS[k:]) < 1e-14)


@pytest.mark.parametrize("m", [1, 5, 17])
def test_truncation(small_sb, m):
    psi = _normalised_psi(small_sb, 12)
    for side in (0, 1):
        tr = OR.truncate(small_sb, psi, side, m)
        assert tr["kept"] == min(m, int(np.sum((small_sb["S"] if side == 0 else small_sb["E"])["dim"])))
        assert abs(tr["eps"] - (1 - np.sum(np.where(tr["lam"] < OR.FLOOR, 0, tr["lam"])))) < 1e-12
        for s, W in tr["W"].items():
            assert np.allclose(W.T @ W, np.eye(W.shape[1]), atol=1e-12)
        # the discarded weight is the norm of psi outside the kept space
        pairs, _ = OS.target_pairs(small_sb)
        out = 0.0
        for (i, j, off) in pairs:
            a, b = int(small_sb["S"]["dim"][i]), int(small_sb["E"]["dim"][j])
            P = psi[off:off + a * b].reshape(a, b)
            sec = i if side == 0 else j
            W = tr["W"].get(sec)
            X = P if side == 0 else P.T
            proj = np.zeros_like(X) if W is None else W @ (W.T @ X)
            out += np.sum((X - proj) ** 2)
        assert abs(out - tr["eps"]) < 1e-12


def test_truncation_keeps_all_when_m_exceeds_dim(small_sb):
    psi = _normalised_psi(small_sb, 13)
    n = int(np.sum(small_sb["S"]["dim"]))
    tr = OR.truncate(small_sb, psi, 0, n + 5)
    assert tr["kept"] == n and tr["eps"] == 0.0


def test_tie_break_and_no_split():
    # two sectors (q=0, q=1) with exactly degenerate weights 0.3, 0.3 and 0.2, 0.2
    sb = dict(S=dict(q=np.array([0, 1]), dim=np.array([2, 2])),
              E=dict(q=np.array([0, 1]), dim=np.array([2, 2])), q_target=1, terms=[])
    # pairs: (0,1) then (1,0); Psi blocks diagonal with sqrt weights
    P01 = np.diag([np.sqrt(0.3), np.sqrt(0.2)])
    P10 = np.diag([np.sqrt(0.3), np.sqrt(0.2)])
    psi = np.concatenate([P01.reshape(-1), P10.reshape(-1)])
    tr = OR.truncate(sb, psi, 0, 1)
    assert tr["kept"] == 1 and tr["lam_sec"][0] == 0 and tr["straddle"]
    tr = OR.truncate(sb, psi, 0, 3)
    assert list(tr["lam_sec"]) == [0, 1, 0]
    tr = OR.truncate(sb, psi, 0, 3, no_split=True)
    assert tr["kept"] == 4 and abs(tr["eps"]) < 1e-15
    tr = OR.truncate(sb, psi, 0, 1, no_split=True)
    assert tr["kept"] == 2 and abs(tr["eps"] - 0.4) < 1e-14


def test_basis_change_block_identities():
    """Eq. (4) and the remark after it: for a square orthogonal W the change
    of basis is a similarity (spectra kept, products commute with it); for a
    truncated W, (W^T A W)(W^T B W) != W^T (A B) W while W^T W = 1."""
    rng = np.random.default_rng(3)
    n, k = 12, 5
    A = rng.standard_normal((n, n))
    A = A + A.T
    B = rng.standard_normal((n, n))
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    At = OR.transform_block(A, Q, Q)
    assert np.allclose(np.linalg.eigvalsh(At), np.linalg.eigvalsh(A))
    assert np.allclose(OR.transform_block(A, Q, Q) @ OR.transform_block(B, Q, Q),
                       OR.transform_block(A @ B, Q, Q))
    W = Q[:, :k]
    assert np.allclose(W.T @ W, np.eye(k))
    lhs = OR.transform_block(A, W, W) @ OR.transform_block(B, W, W)
    assert not np.allclose(lhs, OR.transform_block(A @ B, W, W))
    # entry by entry
    Wr, Wc = Q[:, :k], Q[:, 2:2 + 3]
    T = OR.transform_block(B, Wr, Wc)
    for i in range(k):
        for j in range(3):
            assert abs(T[i, j] - sum(Wr[a, i] * B[a, b] * Wc[b, j]
                                     for a in range(n) for b in range(n))) < 1e-12


def _term_matrices(sb):
    """Each term's explicit Kronecker matrix (target rows and columns), built
    from the dense operators term by term."""
    idx = OS.target_indices(sb)
    out = []
    for t in sb["terms"]:
        A = OS.full_operator(t["A"], sb["S"])
        B = OS.full_operator(t["B"], sb["E"])
        out.append((t["c"], np.kron(A, B)[np.ix_(idx, idx)]))
    return out


def test_element_matches_blocks_at_every_entry(small_sb):
    """hpsi_element (the single-entry form used for sampled checks at full
    size) equals hpsi_blocks entry by entry, and its absolute form equals
    sum_k |c_k| (|A_k| (x) |B_k|) |psi| from the explicit Kronecker matrices."""
    pairs, D = OS.target_pairs(small_sb)
    psi = seeded_vector(D, 7)
    y = OS.hpsi_blocks(small_sb, psi)
    yabs = sum(abs(c) * (np.abs(K) @ np.abs(psi)) for c, K in _term_matrices(small_sb))
    dS, dE = small_sb["S"]["dim"], small_sb["E"]["dim"]
    scale = np.max(np.abs(yabs))
    for (i, j, off) in pairs:
        a, b = int(dS[i]), int(dE[j])
        for m in range(a):
            for n in range(b):
                e = off + m * b + n
                assert abs(OS.hpsi_element(small_sb, psi, i, j, m, n) - y[e]) <= 1e-13 * scale
                got = OS.hpsi_element(small_sb, np.abs(psi), i, j, m, n, absolute=True)
                assert abs(got - yabs[e]) <= 1e-13 * scale


def test_abs_description_bounds_the_product(small_sb):
    """hpsi_blocks(abs_description(sb), |psi|) -- the tolerance scale of the
    GPU parity tests -- is sum_k |c_k| (|A_k| (x) |B_k|) |psi| from the
    explicit Kronecker matrices, and bounds |H psi| entry by entry (triangle
    inequality); every block of the description is the elementwise absolute
    value of the original's."""
    _, D = OS.target_pairs(small_sb)
    psi = seeded_vector(D, 8)
    ab = OS.abs_description(small_sb)
    for t, ta in zip(small_sb["terms"], ab["terms"]):
        assert ta["c"] == abs(t["c"])
        for side in ("A", "B"):
            if t[side] is None:
                assert ta[side] is None
                continue
            assert ta[side]["delta"] == t[side]["delta"]
            for (r, c, blk), (r2, c2, blk2) in zip(t[side]["blocks"], ta[side]["blocks"]):
                assert (r, c) == (r2, c2) and np.array_equal(blk2, np.abs(blk))
    s = OS.hpsi_blocks(ab, np.abs(psi))
    want = sum(abs(c) * (np.abs(K) @ np.abs(psi)) for c, K in _term_matrices(small_sb))
    assert np.max(np.abs(s - want)) <= 1e-13 * np.max(want)
    assert np.all(np.abs(OS.hpsi_blocks(small_sb, psi)) <= s * (1 + 1e-12) + 1e-300)
