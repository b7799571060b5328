"""Host FP64 eigensolvers of the library (the landmark factor's full solver and
the top-k solver behind the PCA basis) against LAPACK's eigh.

The C++ source is compiled here with the system C++ compiler into a small
shared library with a C wrapper (no GPU needed).  Bars: eigenvalues within
1e-12 of the largest; residual |A v - lambda v| within 1e-12 |A|; columns
orthonormal to 1e-12; vectors of eigenvalues isolated by a relative gap of
1e-6 equal to LAPACK's up to sign (|v . v_ref| >= 1 - 1e-10); a cluster's
vectors span LAPACK's invariant subspace of the whole cluster.
"""
import ctypes as ct
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EIG_SRC = os.path.join(ROOT, "paper_1901_06112_amd", "csrc", "eig.cpp")

WRAPPER = r"""
namespace nkf {
int sym_eig(int n, const double *A, double *w, double *V);
int sym_eig_top(int n, const double *A, int k, double *w, double *V);
}
extern "C" int t_sym_eig(int n, const double *A, double *w, double *V) { return nkf::sym_eig(n, A, w, V); }
extern "C" int t_sym_eig_top(int n, const double *A, int k, double *w, double *V) {
  return nkf::sym_eig_top(n, A, k, w, V);
}
"""


@pytest.fixture(scope="module")
def eiglib(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("eig")
    wrap = d / "wrap.cpp"
    wrap.write_text(WRAPPER)
    so = d / "libeigt.so"
    subprocess.run([cxx, "-O2", "-std=c++17", "-shared", "-fPIC", "-o", str(so), EIG_SRC, str(wrap)],
                   check=True, capture_output=True)
    lib = ct.CDLL(str(so))
    P = ct.c_void_p
    lib.t_sym_eig.argtypes = [ct.c_int, P, P, P]
    lib.t_sym_eig_top.argtypes = [ct.c_int, P, ct.c_int, P, P]
    return lib


def _ptr(a):
    return a.ctypes.data_as(ct.c_void_p)


def _full(lib, A):
    n = A.shape[0]
    w, V = np.zeros(n), np.zeros((n, n))
    assert lib.t_sym_eig(n, _ptr(A), _ptr(w), _ptr(V)) == 0
    return w, V


def _top(lib, A, k):
    n = A.shape[0]
    w, V = np.zeros(k), np.zeros((n, k))
    assert lib.t_sym_eig_top(n, _ptr(A), k, _ptr(w), _ptr(V)) == 0
    return w, V


def _check(A, w, V, wref, Vref, k):
    """w, V: the k largest pairs, ascending; wref, Vref: LAPACK's full result."""
    n = A.shape[0]
    scale = np.abs(wref).max()
    np.testing.assert_allclose(w, wref[n - k:], rtol=0, atol=1e-12 * scale)
    anorm = np.abs(A).sum(1).max()
    assert np.abs(A @ V - V * w).max() <= 1e-12 * anorm
    assert np.abs(V.T @ V - np.eye(k)).max() <= 1e-12
    for j in range(k):
        c = n - k + j
        gap = min([abs(wref[c] - wref[i]) for i in (c - 1, c + 1) if 0 <= i < n] or [np.inf])
        if gap > 1e-6 * scale:
            assert abs(V[:, j] @ Vref[:, c]) >= 1 - 1e-10
    # every computed vector lies in the span of LAPACK's vectors for
    # eigenvalues within 1e-8 |A| of its own
    for j in range(k):
        near = np.abs(wref - w[j]) <= 1e-8 * scale
        proj = Vref[:, near] @ (Vref[:, near].T @ V[:, j])
        assert np.linalg.norm(V[:, j] - proj) <= 1e-8


def _spd(n, seed):
    B = np.random.default_rng(seed).normal(size=(n, n))
    return B @ B.T


def _lowrank_plus_identity(n, rank, seed):
    U = np.random.default_rng(seed).normal(size=(n, rank))
    return 100.0 * U @ U.T + np.eye(n)


def _decay(n, seed):
    Q, _ = np.linalg.qr(np.random.default_rng(seed).normal(size=(n, n)))
    lam = 1e6 * 0.7 ** np.arange(n) + 50.0
    return (Q * lam) @ Q.T


def _gauss_gram(n, sr, seed):
    c = np.random.default_rng(seed).uniform(0, 255, size=(n, 3))
    d2 = ((c[:, None, :] - c[None, :, :]) ** 2).sum(-1)
    return np.exp(-d2 / (2 * sr * sr))


@pytest.mark.parametrize("name,A,k", [
    ("spd147", _spd(147, 1), 25),
    ("spd147_all", _spd(147, 2), 147),
    ("lowrank_plus_I", _lowrank_plus_identity(147, 10, 3), 25),  # 137-fold eigenvalue 1
    ("decay", _decay(75, 4), 25),
    ("tiny", _spd(3, 5), 3),
    ("one", np.array([[2.5]]), 1),
    ("diag_ties", np.diag([3.0, 1.0, 3.0, 2.0, 3.0]), 4),
])
def test_top_k_solver_matches_lapack(eiglib, name, A, k):
    A = np.ascontiguousarray(A, np.float64)
    wref, Vref = np.linalg.eigh(A)
    w, V = _top(eiglib, A, k)
    _check(A, w, V, wref, Vref, k)


@pytest.mark.parametrize("n,sr", [(32, 40.0), (128, 121.0), (64, 1e4)])
def test_full_solver_matches_lapack(eiglib, n, sr):
    """The landmark Gram matrix of Eq. (defA): eigenvalues spanning many decades."""
    A = _gauss_gram(n, sr, n)
    wref, Vref = np.linalg.eigh(A)
    w, V = _full(eiglib, A)
    _check(A, w, V, wref, Vref, n)


def test_top_k_rejects_bad_k(eiglib):
    A = _spd(5, 6)
    w, V = np.zeros(6), np.zeros((5, 6))
    assert eiglib.t_sym_eig_top(5, _ptr(A), 0, _ptr(w), _ptr(V)) == -1
    assert eiglib.t_sym_eig_top(5, _ptr(A), 6, _ptr(w), _ptr(V)) == -1
