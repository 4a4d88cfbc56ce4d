"""CPU checks of the C-ABI library: exports, the host plan and host utilities.

No device compute is called: superblocks are built with a NULL context,
which builds the host plan only.
"""
import ctypes as C
import subprocess

import numpy as np
import pytest

from oracle import superblock as OS
from paper_0902_3185_amd import _lib
from paper_0902_3185_amd.superblock import Superblock
from workloads import WORKLOADS, make_superblock, workload_superblock


def test_every_declared_symbol_is_exported():
    declared = _lib.declared_symbols()
    assert len(declared) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if l.strip()}
    missing = [s for s in declared if s not in exported]
    assert not missing, missing
    L = _lib.lib()
    for s in declared:
        assert hasattr(L, s)


@pytest.mark.parametrize("name", list(WORKLOADS))
def test_host_plan_layout_matches_oracle(name):
    desc = workload_superblock(name, m=48)
    sb = Superblock(desc, prec="fp64", ctx=None)
    pairs, D = OS.target_pairs(desc)
    assert sb.D == D
    assert list(sb.s_sec) == [p[0] for p in pairs]
    assert list(sb.e_sec) == [p[1] for p in pairs]
    assert list(sb.offsets) == [p[2] for p in pairs]
    st = sb.stats()
    assert st["ntiles"] > 0 and st["flops_exec"] >= st["flops_alg"] * 0.5


def test_full_size_headline_layout():
    desc = workload_superblock("hubbard_L64_U4_m512")
    sb = Superblock(desc, prec="fp32", ctx=None)
    pairs, D = OS.target_pairs(desc)
    assert sb.D == D and len(sb.s_sec) == len(pairs)


def _tiny():
    return make_superblock("spin", 8, 4, "chain", 1.0, seed=1)


def _err(desc, prec="fp64"):
    with pytest.raises(_lib.DmrgError) as e:
        Superblock(desc, prec=prec, ctx=None)
    return e.value.name


def test_error_q_not_increasing():
    d = _tiny()
    d["S"]["q"] = d["S"]["q"][::-1].copy()
    assert _err(d) == "DMRG_E_QN"


def test_error_block_breaks_delta():
    d = _tiny()
    t = next(t for t in d["terms"] if t["A"] is not None and t["A"]["delta"] != 0)
    r, c, b = t["A"]["blocks"][0]
    t["A"]["blocks"][0] = (c, c, np.zeros((b.shape[1], b.shape[1])))
    assert _err(d) == "DMRG_E_QN"


def test_error_term_not_neutral():
    d = _tiny()
    t = next(t for t in d["terms"] if t["A"] is not None and t["B"] is not None
             and t["A"]["delta"] != 0)
    t["B"] = None
    assert _err(d) == "DMRG_E_QN"


def test_error_empty_target():
    d = _tiny()
    d["q_target"] = 10 ** 9
    assert _err(d) == "DMRG_E_QN"


def test_error_bad_dimension():
    d = _tiny()
    d["S"]["dim"] = d["S"]["dim"].copy()
    d["S"]["dim"][0] = 0
    assert _err(d) == "DMRG_E_SHAPE"


def test_error_dense_both_sides():
    d = make_superblock("spin", 12, 6, "ladder", 1.2, seed=1)
    t = next(t for t in d["terms"] if t["A"] is not None and t["B"] is not None)
    dense = next(tt for tt in d["terms"] if tt["A"] is not None and tt["B"] is None)
    t2 = dict(c=1.0, A=dense["A"], B=next(tt for tt in d["terms"]
                                        if tt["A"] is None and tt["B"] is not None)["B"], group=0)
    d["terms"].append(t2)
    assert t is not None
    assert _err(d) == "DMRG_E_UNSUPPORTED"


def test_device_calls_need_a_context():
    import torch
    sb = Superblock(_tiny(), prec="fp64", ctx=None)
    st = _lib.lib().dmrg_hpsi(sb.handle, C.c_void_p(16), C.c_void_p(32), 1.0, 0.0)
    assert _lib.STATUS[st] == "DMRG_E_DEVICE"
    assert torch is not None


def test_host_sym_eigen_matches_numpy():
    rng = np.random.default_rng(0)
    for n in (1, 2, 3, 17, 64, 150):
        X = rng.standard_normal((n, n))
        A = X + X.T
        if n >= 17:   # add an exactly degenerate pair and a zero block
            Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
            ev = np.linspace(-1, 1, n)
            ev[3] = ev[4]
            ev[:2] = 0.0
            A = (Q * ev) @ Q.T
            A = 0.5 * (A + A.T)
        a = np.ascontiguousarray(A.copy())
        w = np.zeros(n)
        _lib.check(_lib.lib().dmrg_host_sym_eigen(n, a.ctypes.data_as(C.POINTER(C.c_double)),
                                                  w.ctypes.data_as(C.POINTER(C.c_double))))
        wr = np.linalg.eigvalsh(A)
        scale = max(1.0, np.abs(wr).max())
        assert np.allclose(w, wr, atol=1e-13 * scale * n)
        V = a
        assert np.allclose(V.T @ V, np.eye(n), atol=1e-12 * n)
        assert np.allclose(A @ V, V * w[None, :], atol=1e-12 * scale * n)


def test_host_sym_eigen_every_small_size():
    """Every size from 1 to 40 (the Householder passes take rows in pairs
    and columns four at a time, so every parity of the row count and every
    remainder of the column loop is met), against NumPy's eigenvalues and the
    eigen-equation itself."""
    rng = np.random.default_rng(3)
    for n in range(1, 41):
        X = rng.standard_normal((n, n))
        A = X @ X.T / n + np.diag(rng.standard_normal(n))
        a = np.ascontiguousarray(A.copy())
        w = np.zeros(n)
        _lib.check(_lib.lib().dmrg_host_sym_eigen(n, a.ctypes.data_as(C.POINTER(C.c_double)),
                                                  w.ctypes.data_as(C.POINTER(C.c_double))))
        scale = np.abs(np.linalg.eigvalsh(A)).max()
        assert np.allclose(w, np.linalg.eigvalsh(A), atol=1e-13 * n * scale), n
        assert np.allclose(a.T @ a, np.eye(n), atol=1e-13 * n), n
        assert np.allclose(A @ a, a * w[None, :], atol=1e-13 * n * scale), n


def test_host_sym_eigen_rank_deficient_density_matrices():
    """rho = Psi Psi^T of rank r < n (the untruncated small blocks of a run),
    with its null space at rounding level: all eigenpairs, no stall."""
    rng = np.random.default_rng(7)
    for n, r in ((64, 20), (150, 30), (256, 64), (97, 1)):
        X = rng.standard_normal((n, r)) * np.exp(-0.4 * np.arange(r))[None, :]
        A = X @ X.T
        A /= np.trace(A)
        a = np.ascontiguousarray(A.copy())
        w = np.zeros(n)
        _lib.check(_lib.lib().dmrg_host_sym_eigen(n, a.ctypes.data_as(C.POINTER(C.c_double)),
                                                  w.ctypes.data_as(C.POINTER(C.c_double))))
        wr = np.linalg.eigvalsh(A)
        assert np.allclose(w, wr, atol=1e-14 * n)
        assert np.allclose(a.T @ a, np.eye(n), atol=1e-12 * n)
        assert np.allclose(A @ a, a * w[None, :], atol=1e-14 * n)


def test_host_sym_eigen_columns_near_underflow():
    """Householder columns whose entries sit near the underflow threshold (the
    trailing rounding-level part of a rank-one density matrix decays there):
    the reflector must be formed on the scaled column."""
    rng = np.random.default_rng(11)
    for n, k in ((40, 20), (87, 3), (130, 1)):
        X = rng.standard_normal((k, k))
        Y = rng.standard_normal((n - k, n - k))
        A = np.zeros((n, n))
        A[:k, :k] = 1e-3 * (X @ X.T)
        A[k:, k:] = 1e-158 * (Y @ Y.T)
        a = np.ascontiguousarray(A.copy())
        w = np.zeros(n)
        _lib.check(_lib.lib().dmrg_host_sym_eigen(n, a.ctypes.data_as(C.POINTER(C.c_double)),
                                                  w.ctypes.data_as(C.POINTER(C.c_double))))
        wr = np.linalg.eigvalsh(A)
        assert np.all(np.isfinite(w)) and np.all(np.isfinite(a))
        assert np.allclose(w, wr, atol=1e-14 * n * np.abs(wr).max())
        assert np.allclose(a.T @ a, np.eye(n), atol=1e-12 * n)


def test_host_tridiag_lowest():
    rng = np.random.default_rng(1)
    for n in (1, 2, 5, 40, 300):
        a = rng.standard_normal(n)
        b = rng.standard_normal(max(n - 1, 0))
        T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
        th = C.c_double()
        u = np.zeros(n)
        bb = b if n > 1 else np.zeros(1)
        _lib.check(_lib.lib().dmrg_host_tridiag_lowest(
            n, a.ctypes.data_as(C.POINTER(C.c_double)), bb.ctypes.data_as(C.POINTER(C.c_double)),
            C.byref(th), u.ctypes.data_as(C.POINTER(C.c_double))))
        w, V = np.linalg.eigh(T)
        assert abs(th.value - w[0]) < 1e-13 * max(1, abs(w).max())
        assert abs(abs(np.dot(u, V[:, 0])) - 1) < 1e-10
        assert np.linalg.norm(T @ u - th.value * u) < 1e-12 * max(1, abs(w).max())
