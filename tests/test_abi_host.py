"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every symbol of include/nkf.h, and its host-only routines -- the seeding draw,
the spatial taps and the FP64 landmark factor -- agree with the oracle and
with LAPACK.  No device compute is called here."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

from oracle import exact, nystrom, seeding
from paper_1901_06112_amd import nkf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    src = open(os.path.join(ROOT, "include", "nkf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nkf_[a-z_]+)\s*\(", src)))


def test_library_exports_every_header_symbol():
    lib = nkf.load_library()
    syms = _header_symbols()
    assert len(syms) >= 15
    assert sorted(nkf.EXPORTS) == syms
    for s in syms:
        assert hasattr(lib, s), s
    assert "gfx950" in nkf.version()


def test_seed_indices_match_oracle_draw():
    # the last two: the PCA patch sample (65536 draws), the first of them a full shuffle
    for N, r, s in [(100, 100, 0), (4194304, 32, 2), (65536, 16, 1), (262144, 64, 12345678901234567),
                    (70000, 65536, 3), (1 << 20, 65536, 1004)]:
        np.testing.assert_array_equal(nkf.seed_indices(N, r, s), seeding.distinct_indices(N, r, s))


def test_spatial_taps_match_oracle():
    for radius, ss, kind in [(-1, 3.0, "gaussian"), (15, 5.0, "gaussian"), (10, 1.0, "box"), (0, 2.0, "gaussian")]:
        S, taps = nkf.spatial_taps(radius, ss, kind)
        assert S == (radius if radius >= 0 else int(np.ceil(3 * ss)))
        np.testing.assert_allclose(taps, exact.spatial_taps(ss, S, kind).astype(np.float32), rtol=0, atol=0)


def test_spatial_taps_radius_limit():
    with pytest.raises(nkf.NkfError) as ei:
        nkf.spatial_taps(-1, 6.0, "gaussian")  # ceil(18) > 16
    assert ei.value.status == nkf.NKF_ERR_UNSUPPORTED


def test_recursive_gaussian_has_no_taps():
    # the recursive filter is not a truncated window: asking for its taps is refused
    with pytest.raises(nkf.NkfError) as ei:
        nkf.spatial_taps(-1, 2.0, "recursive")
    assert ei.value.status == nkf.NKF_ERR_UNSUPPORTED


def _check_factor(c, sr, tau=1e-10):
    Q, al, F, reff = nkf.landmark_factor(c, sr, tau)
    A = nystrom.landmark_gram(c, sr)
    ref = np.linalg.eigvalsh(A)
    np.testing.assert_allclose(al, ref, rtol=0, atol=1e-12 * max(1.0, abs(ref).max()))
    np.testing.assert_allclose(Q @ np.diag(al) @ Q.T, A, rtol=0, atol=1e-12 * A.shape[0])
    np.testing.assert_allclose(Q.T @ Q, np.eye(len(al)), rtol=0, atol=1e-12 * A.shape[0])
    # F F^T = A^+ on the kept subspace
    a_or, W_or = nystrom.landmark_eig(c, sr, tau)
    assert reff == len(a_or)
    pinv = (W_or / a_or) @ W_or.T
    np.testing.assert_allclose(F @ F.T, pinv, rtol=1e-8, atol=1e-8 * np.abs(pinv).max())
    return reff


def test_landmark_factor_random_and_gaussian_gram():
    rng = np.random.default_rng(0)
    for r, D, sr in [(16, 3, 30.0), (32, 3, 40.0), (64, 128, 0.3 * 10), (128, 147, 121.24), (7, 2, 5.0)]:
        c = rng.uniform(0, 255 if D < 100 else 1, (r, D))
        if D >= 100:
            c = c * 2.0
        _check_factor(c, sr)


def test_landmark_factor_rank_deficient():
    rng = np.random.default_rng(1)
    c = rng.uniform(0, 255, (10, 3))
    c[5] = c[2]                        # coincident landmarks: A singular
    c[7] = c[2]
    assert _check_factor(c, 30.0) == 8
    assert _check_factor(c, 1e7) == 1  # sigma_r -> inf: rank one
    Q, al, F, reff = nkf.landmark_factor(c, float("inf"))
    assert reff == 1 and abs(al[-1] - 10.0) < 1e-12


def test_landmark_factor_single_and_errors():
    Q, al, F, reff = nkf.landmark_factor(np.array([[1.0, 2.0, 3.0]]), 10.0)
    assert reff == 1 and al[0] == 1.0 and abs(F[0, 0]) == 1.0
    with pytest.raises(nkf.NkfError) as ei:
        nkf.landmark_factor(np.zeros((3, 2)), -1.0)
    assert ei.value.status == nkf.NKF_ERR_INVALID_ARG
    with pytest.raises(nkf.NkfError):
        nkf.landmark_factor(np.zeros((300, 2)), 1.0)


def test_seed_indices_errors():
    with pytest.raises(nkf.NkfError):
        nkf.seed_indices(5, 6, 0)
