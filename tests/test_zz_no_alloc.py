"""dmrg_hpsi_noalloc (the product with its temporaries in the library's fixed
device scratch, allocating nothing) against dmrg_hpsi, through the C ABI.

Both entry points run the same kernels on the same inputs, so their outputs
must agree bit for bit; both are also checked against the oracle to the
product's tolerance.  Two calls in a row, the second on a smaller
superblock, show that what the first call left in the scratch does not leak
into the second.
"""
import ctypes as C

import numpy as np
import pytest

from oracle import superblock as OS
from workloads import seeded_vector, workload_superblock

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-14, "fp32": 4e-6, "bf16x3": 5e-5}


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_0902_3185_amd.superblock import Context
    assert torch.cuda.is_available()
    return Context(0)


def _dev(x):
    import torch
    return torch.tensor(np.asarray(x), dtype=torch.float64, device="cuda")


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _call(fn, sb, psi, y, alpha, beta):
    from paper_0902_3185_amd import _lib
    _lib.check(getattr(_lib.lib(), fn)(sb.handle, C.c_void_p(psi.data_ptr()), C.c_void_p(y.data_ptr()),
                                        float(alpha), float(beta)))


CASES = [("fp32", 0), ("bf16x3", 0), ("fp64", 0), ("fp32", 1), ("bf16x3", 1)]


@pytest.mark.parametrize("prec,variant", CASES, ids=[f"{p}-v{v}" for p, v in CASES])
def test_noalloc_matches_hpsi_on_two_calls(ctx, prec, variant):
    """Variant 1 (the macro-tile kernel) also keeps its partial tiles and
    tile counters in the scratch; the ladder superblock shares most of its
    tiles between workgroups.  Variant 0 runs on the physical headline
    superblock."""
    from paper_0902_3185_amd.superblock import Superblock
    first = ("ladder_2x32_m1024", None, 0) if variant else ("hubbard_L64_U4_m512_physical", None, 0)
    for name, m, seed in [first, ("heisenberg_L100_m256", 64, 1)]:
        desc = workload_superblock(name, m=m, seed=seed)
        sb = Superblock(desc, prec=prec, ctx=ctx)
        if variant:
            sb.set_variant(variant)
        psi = seeded_vector(sb.D, 71)
        y0 = seeded_vector(sb.D, 72)
        ya, yb = _dev(y0), _dev(y0)
        _call("dmrg_hpsi", sb, _dev(psi), ya, 0.7, -0.3)
        _call("dmrg_hpsi_noalloc", sb, _dev(psi), yb, 0.7, -0.3)
        a, b = _host(ya), _host(yb)
        assert np.array_equal(a, b), (name, prec)
        ref = 0.7 * OS.hpsi_blocks(desc, psi) - 0.3 * y0
        scale = np.linalg.norm(OS.hpsi_blocks(OS.abs_description(desc), np.abs(psi)))
        assert np.linalg.norm(b - ref) <= TOL[prec] * scale, (name, prec)
        sb.close()


def test_noalloc_argument_errors(ctx):
    from paper_0902_3185_amd import _lib
    from paper_0902_3185_amd.superblock import Superblock
    desc = workload_superblock("heisenberg_L16_m32", seed=0)
    sb = Superblock(desc, prec="fp32", ctx=ctx)
    x = _dev(seeded_vector(sb.D, 1))
    st = _lib.lib().dmrg_hpsi_noalloc(sb.handle, C.c_void_p(x.data_ptr()), C.c_void_p(x.data_ptr()), 1.0, 0.0)
    assert _lib.STATUS[st] == "DMRG_E_ARG"
    st = _lib.lib().dmrg_hpsi_noalloc(sb.handle, None, C.c_void_p(x.data_ptr()), 1.0, 0.0)
    assert _lib.STATUS[st] == "DMRG_E_ARG"
