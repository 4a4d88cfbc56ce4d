"""GPU parity of the superblock product and its adjoint against the oracle.

Both sides get the same seeded superblocks and vectors (workloads).  Every
entry is held to the rounding bound of fp_bounds: (n_i + 10) u (|H||psi|)_i
for an entry summing n_i nonzero products (plus the split remainder
3.01 * 2^-16 and three additions per product for the BF16 split).  The norm
of the error is also held to a tolerance relative to || |H| |psi| ||: FP64 products carry the rounding of
a K-term FP64 sum (K <= ~600), bounded here by 1e-14; FP32 products round
the operands once (2^-24 each) and accumulate K terms in FP32, which for
random-sign rounding errors is ~(2 + sqrt(K)) 2^-24 <= 1.6e-6 at K = 600;
the test allows 4e-6.  BF16 hi/lo x3 keeps hi*hi + hi*lo + lo*hi of operands
split into two bf16 parts (8 significant bits each), leaving ~2^-16 relative
per product before FP32 accumulation; the test allows 5e-5.
"""
import numpy as np
import pytest

from oracle import superblock as OS
from workloads import WORKLOADS, seeded_vector, workload_superblock
from workloads.superblocks import FIXTURES

import fp_bounds as FB

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-14, "fp64_plain": 1e-14, "fp32": 4e-6, "bf16x3": 5e-5}

# reduced sizes: several 32-wide tiles per block and ragged tails
CASES = [("heisenberg_L16_m32", None), ("heisenberg_L100_m256", 64),
         ("hubbard_L64_U4_m512", 96), ("ladder_2x32_m1024", 80), ("j1j2_L64_m256", 64)]


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


def _scale(desc, psi):
    return np.linalg.norm(OS.hpsi_blocks(OS.abs_description(desc), np.abs(psi)))


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "fp64_plain"])
@pytest.mark.parametrize("name,m", CASES, ids=[c[0] for c in CASES])
def test_hpsi_parity(ctx, name, m, prec):
    from paper_0902_3185_amd.superblock import Superblock
    desc = workload_superblock(name, m=m, seed=1)
    sb = Superblock(desc, prec=prec, ctx=ctx)
    psi = seeded_vector(sb.D, 11)
    y0 = seeded_vector(sb.D, 12)
    ref = 0.7 * OS.hpsi_blocks(desc, psi) - 0.3 * y0
    y = _host(sb.hpsi(_dev(psi), _dev(y0), alpha=0.7, beta=-0.3))
    err = np.linalg.norm(y - ref)
    assert err <= TOL[prec] * _scale(desc, psi), (name, prec, err)
    # entry by entry: 0.7 times the bound of H psi, plus the roundings of the
    # FP64 update alpha v + beta y (|v| <= s)
    s, bound = FB.product_bound(desc, psi, prec)
    ebound = 0.7 * bound + 4 * 2.0 ** -53 * (0.7 * s + 0.3 * np.abs(y0))
    assert np.all(np.abs(y - ref) <= ebound), (name, prec)
    # beta = 0 must not read y (fill it with NaN first)
    import torch
    yn = torch.full((sb.D,), float("nan"), dtype=torch.float64, device="cuda")
    y2 = _host(sb.hpsi(_dev(psi), yn, alpha=1.0, beta=0.0))
    assert np.all(np.isfinite(y2))
    assert np.linalg.norm(y2 - OS.hpsi_blocks(desc, psi)) <= TOL[prec] * _scale(desc, psi)


FULL_CASES = [(p, 0) for p in ("fp64", "fp32", "bf16x3", "fp64_plain")] + [("fp32", 1), ("bf16x3", 1)]


@pytest.mark.parametrize("prec,variant", FULL_CASES, ids=[f"{p}-v{v}" for p, v in FULL_CASES])
@pytest.mark.parametrize("name", list(WORKLOADS) + list(FIXTURES))
def test_full_size_elementwise(ctx, name, prec, variant):
    """Every workload at its full size (the centre superblocks the benchmark
    times, same launch paths: the 32 x 32 tile kernel and the 64 x 64
    macro-tile kernel), the stored physical Hubbard superblock included:
    every entry of H psi within its rounding bound, and the error norm
    within the aggregate tolerance."""
    from paper_0902_3185_amd.superblock import Superblock
    desc = workload_superblock(name, seed=0)
    sb = Superblock(desc, prec=prec, ctx=ctx)
    if variant:
        sb.set_variant(variant)
    psi = seeded_vector(sb.D, 21)
    print(f"full-size product {name} {prec} variant {variant} D={sb.D}", flush=True)
    y = _host(sb.hpsi(_dev(psi)))
    ref = OS.hpsi_blocks(desc, psi)
    s, bound = FB.product_bound(desc, psi, prec)
    err = np.abs(y - ref)
    over = np.flatnonzero(err > bound)
    assert over.size == 0, (name, prec, over[:5], err[over[:5]], bound[over[:5]])
    assert np.linalg.norm(y - ref) <= TOL[prec] * np.linalg.norm(s), (name, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_deterministic_and_hermitian(ctx, prec):
    from paper_0902_3185_amd.superblock import Superblock
    desc = workload_superblock("ladder_2x32_m1024", m=64, seed=2)
    sb = Superblock(desc, prec=prec, ctx=ctx)
    x = seeded_vector(sb.D, 1)
    yv = seeded_vector(sb.D, 2)
    h1 = _host(sb.hpsi(_dev(x)))
    h2 = _host(sb.hpsi(_dev(x)))
    assert np.array_equal(h1, h2)
    hy = _host(sb.hpsi(_dev(yv)))
    lhs, rhs = np.dot(yv, h1), np.dot(hy, x)
    tol = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 1e-4}[prec]
    assert abs(lhs - rhs) <= tol * (np.linalg.norm(h1) * np.linalg.norm(yv))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name,m", [("j1j2_L64_m256", 48), ("ladder_2x32_m1024", 48),
                                    ("hubbard_L64_U4_m512", 64), ("j1j2_L64_m256", None),
                                    ("hubbard_L64_U4_m512", None), ("hubbard_L64_U4_m512_physical", None)])
def test_adjoint_parity(ctx, name, m, prec):
    from paper_0902_3185_amd.superblock import Superblock
    desc = workload_superblock(name, m=m, seed=3)
    sb = Superblock(desc, prec=prec, ctx=ctx)
    psi = seeded_vector(sb.D, 31)
    g = seeded_vector(sb.D, 32)
    gp_ref, gc_ref = OS.hpsi_adjoint_blocks(desc, psi, g)
    gp, gc = sb.adjoint(_dev(psi), _dev(g))
    gp = _host(gp)
    s_t, gp_bound, gc_bound = FB.adjoint_bound(desc, psi, g, prec)
    assert np.linalg.norm(gp - gp_ref) <= TOL[prec] * np.linalg.norm(s_t)
    assert np.all(np.abs(gp - gp_ref) <= gp_bound)
    assert np.all(np.abs(np.asarray(gc) - gc_ref) <= gc_bound), (np.abs(gc - gc_ref), gc_bound)


def test_set_coeffs_is_linear(ctx):
    from paper_0902_3185_amd.superblock import Superblock
    desc = workload_superblock("j1j2_L64_m256", m=48, seed=4)
    sb = Superblock(desc, prec="fp64", ctx=ctx)
    psi = seeded_vector(sb.D, 41)
    c = np.array([t["c"] for t in desc["terms"]])
    c2 = c * np.linspace(0.5, 1.5, len(c))
    sb.set_coeffs(c2)
    y = _host(sb.hpsi(_dev(psi)))
    ref = OS.hpsi_blocks(desc, psi, coeffs=c2)
    assert np.linalg.norm(y - ref) <= 1e-14 * _scale(desc, psi) * 2


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "fp64_plain"])
def test_set_coeffs_between_products(ctx, prec):
    """New coefficients apply to the products enqueued after them and not to
    the ones before, with no synchronisation in between; the adjoint too."""
    import torch
    from paper_0902_3185_amd.superblock import Superblock
    desc = workload_superblock("hubbard_L64_U4_m512", m=96, seed=4)
    sb = Superblock(desc, prec=prec, ctx=ctx)
    psi = _dev(seeded_vector(sb.D, 42))
    g = _dev(seeded_vector(sb.D, 43))
    c1 = np.array([t["c"] for t in desc["terms"]])
    c2 = c1 * np.linspace(-1.5, 2.0, len(c1))
    outs = []
    for c in (c1, c2, c1, c2):
        sb.set_coeffs(c)
        outs.append(torch.clone(sb.hpsi(psi)))
    gp2, gc2 = sb.adjoint(psi, g)
    torch.cuda.synchronize()
    p = psi.cpu().numpy()
    for c, y in zip((c1, c2, c1, c2), outs):
        d = dict(desc, terms=[dict(t, c=float(ck)) for t, ck in zip(desc["terms"], c)])
        ref = OS.hpsi_blocks(d, p)
        _, bound = FB.product_bound(d, p, prec)
        assert np.all(np.abs(y.cpu().numpy() - ref) <= bound)
    if prec in ("fp64", "fp32"):
        d2 = dict(desc, terms=[dict(t, c=float(ck)) for t, ck in zip(desc["terms"], c2)])
        gp_ref, gc_ref = OS.hpsi_adjoint_blocks(d2, p, g.cpu().numpy())
        _, gp_bound, gc_bound = FB.adjoint_bound(d2, p, g.cpu().numpy(), prec)
        assert np.all(np.abs(_host(gp2) - gp_ref) <= gp_bound)
        assert np.all(np.abs(np.asarray(gc2) - gc_ref) <= gc_bound)


def test_argument_errors(ctx):
    from paper_0902_3185_amd import _lib
    from paper_0902_3185_amd.superblock import Superblock
    desc = workload_superblock("heisenberg_L16_m32", seed=0)
    sb = Superblock(desc, prec="fp64", ctx=ctx)
    x = _dev(seeded_vector(sb.D, 1))
    import ctypes as C
    st = _lib.lib().dmrg_hpsi(sb.handle, C.c_void_p(x.data_ptr()), C.c_void_p(x.data_ptr()), 1.0, 0.0)
    assert _lib.STATUS[st] == "DMRG_E_ARG"
    with pytest.raises(ValueError):
        sb.hpsi(_dev(np.zeros(sb.D + 1)))


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("name,m", [("hubbard_L64_U4_m512", 96), ("ladder_2x32_m1024", 80),
                                    ("heisenberg_L100_m256", None)])
def test_kernel_variants_and_autotune(ctx, name, m, prec):
    """Every variant of the fused kernel is within tolerance of the oracle and
    repeatable; the autotuner picks one of them, whose bits later products
    reproduce; an unknown variant is an argument error."""
    from paper_0902_3185_amd.superblock import Superblock
    desc = workload_superblock(name, m=m, seed=5)
    sb = Superblock(desc, prec=prec, ctx=ctx)
    psi = seeded_vector(sb.D, 51)
    ref = OS.hpsi_blocks(desc, psi)
    outs = []
    for v in range(64):
        try:
            sb.set_variant(v)
        except Exception:
            break
        y = _host(sb.hpsi(_dev(psi)))
        assert np.array_equal(y, _host(sb.hpsi(_dev(psi)))), v
        assert np.linalg.norm(y - ref) <= TOL[prec] * _scale(desc, psi), v
        outs.append(y)
    assert outs
    chosen = sb.autotune(reps=3)
    assert 0 <= chosen < len(outs)
    assert np.array_equal(_host(sb.hpsi(_dev(psi))), outs[chosen])
    with pytest.raises(Exception):
        sb.set_variant(len(outs))


def test_product_in_captured_graph(ctx):
    """Products captured in a hipGraph (through torch) replay to the eager
    result, several times, with eager work and synchronisation between."""
    import torch
    from paper_0902_3185_amd.superblock import Superblock
    desc = workload_superblock("hubbard_L64_U4_m512", m=96, seed=7)
    sb = Superblock(desc, prec="fp32", ctx=ctx)
    psi = _dev(seeded_vector(sb.D, 61))
    ref = _host(sb.hpsi(psi))
    y = torch.empty_like(psi)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ctx.set_stream(side)
        sb.hpsi(psi, y)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    try:
        with torch.cuda.graph(g, stream=side):
            ctx.set_stream(side)
            sb.hpsi(psi, y)
    finally:
        ctx.set_stream(torch.cuda.current_stream())
    for rep in range(4):
        y.fill_(float("nan"))
        sb.hpsi(psi, torch.empty_like(psi))     # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(_host(y), ref), rep


def test_sampled_product_timing(ctx):
    """dmrg_ctx_set_timing(ctx, k): every k-th product launch is event-timed
    and every launch is counted; the sampled launches give a positive time."""
    import ctypes as C
    from paper_0902_3185_amd import _lib
    from paper_0902_3185_amd.superblock import Superblock
    desc = workload_superblock("heisenberg_L16_m32", seed=0)
    sb = Superblock(desc, prec="fp64", ctx=ctx)
    x = _dev(seeded_vector(sb.D, 1))
    y = _dev(np.zeros(sb.D))
    ctx.timing("fp64", reset=True)
    ctx.set_timing(3)
    for _ in range(10):
        sb.hpsi(x, y)
    ms, timed, total = ctx.timing("fp64", reset=True, products=True)
    ctx.set_timing(0)
    assert (timed, total) == (4, 10) and ms > 0.0
    ms, timed, total = ctx.timing("fp64", reset=True, products=True)
    assert (ms, timed, total) == (0.0, 0, 0)
    assert _lib.STATUS[_lib.lib().dmrg_ctx_set_timing(ctx.handle, -1)] == "DMRG_E_ARG"
