"""GPU parity of the basis change (Eq. (4)) against the oracle."""
import numpy as np
import pytest

from oracle import rho as OR
from workloads import seeded_vector

pytestmark = pytest.mark.gpu


def test_transform_blocks_parity():
    import torch
    from paper_0902_3185_amd.superblock import Context
    ctx = Context(0)
    rng = np.random.default_rng(7)
    shapes = [(1, 1, 1, 1), (7, 5, 3, 2), (40, 33, 17, 31), (212, 190, 100, 64), (65, 97, 64, 33)]
    O, W, blocks, want = [], [], [], []
    o_off = w_off = out_off = 0
    for (r, c, kr, kc) in shapes:
        Ob = rng.standard_normal((r, c))
        Wr = np.linalg.qr(rng.standard_normal((r, r)))[0][:, :kr]
        Wc = np.linalg.qr(rng.standard_normal((c, c)))[0][:, :kc]
        blocks.append(dict(o_off=o_off, rows=r, cols=c, wr_off=w_off, kr=kr,
                           wc_off=w_off + r * kr, kc=kc, out_off=out_off))
        O.append(Ob.reshape(-1))
        W += [Wr.reshape(-1), Wc.reshape(-1)]
        want.append(OR.transform_block(Ob, Wr, Wc).reshape(-1))
        o_off += r * c
        w_off += r * kr + c * kc
        out_off += kr * kc
    dO = torch.tensor(np.concatenate(O), device="cuda")
    dW = torch.tensor(np.concatenate(W), device="cuda")
    out = torch.full((out_off,), float("nan"), dtype=torch.float64, device="cuda")
    ctx.transform_blocks(blocks, dO, dW, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ref = np.concatenate(want)
    assert np.all(np.isfinite(got))
    assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
    assert seeded_vector(1, 0) is not None


def test_transform_strided_slices():
    """o_ld / out_ld: a column slice in, a column slice of a wider block out."""
    import torch
    from paper_0902_3185_amd.superblock import Context
    ctx = Context(0)
    rng = np.random.default_rng(8)
    big = rng.standard_normal((37, 90))
    Wr = np.linalg.qr(rng.standard_normal((37, 37)))[0][:, :20]
    Wc = rng.standard_normal((33, 41))
    out_w = 70
    blocks = [dict(o_off=11, rows=37, cols=33, o_ld=90, wr_off=0, kr=20, wc_off=37 * 20, kc=41,
                   out_off=5, out_ld=out_w)]
    dO = torch.tensor(big.reshape(-1), device="cuda")
    dW = torch.tensor(np.concatenate([Wr.reshape(-1), Wc.reshape(-1)]), device="cuda")
    out = torch.zeros(20 * out_w, dtype=torch.float64, device="cuda")
    ctx.transform_blocks(blocks, dO, dW, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ref = np.zeros(20 * out_w)
    R = OR.transform_block(big[:, 11:11 + 33], Wr, Wc)
    for i in range(20):
        ref[5 + i * out_w:5 + i * out_w + 41] = R[i]
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))
