"""CPU-only checks of the C ABI library and of the host factorisation.

No GPU work is launched here: the library is loaded and inspected, and the
host nested-dissection LU is exercised through a small C++ driver that
applies the stored inverted supernode blocks on the CPU in the same level
order the GPU kernels use (tests/cpp/ndfact_check.cpp)."""
import ctypes
import os
import subprocess

import numpy as np
import pytest
import scipy.sparse.linalg as spla

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2008_10275_amd import lrcheb
    if not os.path.exists(lrcheb.LIB_PATH):
        pytest.fail("liblrcheb.so is not built: run __graft_entry__.build()")
    lrcheb.load()
    return lrcheb


def test_library_exports_every_header_symbol(L):
    names = L.header_symbols()
    assert len(names) >= 20
    lib = ctypes.CDLL(L.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # every declared function has a binding signature and vice versa
    assert set(names) == set(L._SIGS)


def test_default_options_match_header_contract(L):
    o = L.default_opts()
    assert o.rank_cap == 20 and o.trunc_tol == 1e-8 and o.res_tol == 1e-8
    assert o.restart == 6 and o.precision == L.LRC_FP64


def test_profile_api_host_side(L):
    L.profile_enable(0)
    t = L.profile_read()
    assert "spmm.f32" in t and "gram.f64" in t and "jacobi.f64" in t
    assert all(v["count"] == 0 for v in t.values())
    with pytest.raises(L.LrcError):
        L.profile_enable(3)


def _build_ndcheck(tmp):
    exe = os.path.join(tmp, "ndcheck")
    src = os.path.join(ROOT, "tests", "cpp", "ndfact_check.cpp")
    lib = os.path.join(ROOT, "paper_2008_10275_amd", "csrc", "host", "ndfact.cpp")
    inc = os.path.join(ROOT, "paper_2008_10275_amd", "csrc", "host")
    subprocess.run(["g++", "-O2", "-fopenmp", "-std=c++17", "-I", inc, src, lib, "-o", exe],
                   check=True, capture_output=True)
    return exe


@pytest.mark.parametrize("leaf", [4, 16])
def test_host_factorisation_solves_mean_preconditioner(tmp_path, leaf):
    from oracle import chebyshev as och
    from workloads import config
    cfg = config("c1")
    P = och.mean_preconditioner(cfg["ops"].K, och.mean_parameters(cfg["d"])).tocsr()
    P.sort_indices()
    n, k = P.shape[0], 3
    R = np.random.default_rng(leaf).standard_normal((n, k))
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(inp, "wb") as f:
        np.array([n, P.nnz], np.int64).tofile(f)
        P.indptr.astype(np.int64).tofile(f)
        P.indices.astype(np.int32).tofile(f)
        P.data.astype(np.float64).tofile(f)
        np.array([k], np.int64).tofile(f)
        R.tofile(f)
    exe = _build_ndcheck(str(tmp_path))
    r = subprocess.run([exe, str(inp), str(out), str(leaf)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    Z = np.fromfile(out, np.float64).reshape(n, k)
    Zs = spla.splu(P.tocsc()).solve(R)
    assert np.linalg.norm(Z - Zs) / np.linalg.norm(Zs) < 1e-12


def test_host_factorisation_reports_zero_pivot(tmp_path):
    # a structurally fine matrix whose first pivot is exactly zero
    import scipy.sparse as sp
    A = sp.csr_matrix(np.array([[0.0, 1.0, 0.0], [1.0, 2.0, 1.0], [0.0, 1.0, 2.0]]))
    A.sort_indices()
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(inp, "wb") as f:
        np.array([3, A.nnz], np.int64).tofile(f)
        A.indptr.astype(np.int64).tofile(f)
        A.indices.astype(np.int32).tofile(f)
        A.data.astype(np.float64).tofile(f)
        np.array([1], np.int64).tofile(f)
        np.ones(3).tofile(f)
    exe = _build_ndcheck(str(tmp_path))
    r = subprocess.run([exe, str(inp), str(out), "1"], capture_output=True, text=True)
    assert '"rc": -4' in r.stdout, r.stdout + r.stderr
