"""The per-atom LNO eigen-routines of the GPU kernel (Sec. II.B, Eq. 20-22), compiled for the
host and checked against LAPACK's general eigensolver (numpy.linalg.eig) and the oracle's LNO
selection: real Schur form, eigenvalues, ranks and the kept span, with complex-conjugate pairs
of eigenvalues kept, dropped and cut through (reading R1 of the design notes)."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle.lno as olno

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LD = 16


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    out = str(tmp_path_factory.mktemp("smalleig") / "libsmall_eig_host.so")
    src = os.path.join(HERE, "small_eig_host.cpp")
    inc = os.path.join(ROOT, "paper_1809_05637_amd", "csrc")
    subprocess.run([gxx, "-O2", "-std=c++17", "-shared", "-fPIC", "-I", inc, src, "-o", out], check=True)
    L = ctypes.CDLL(out)
    P = ctypes.POINTER(ctypes.c_double)
    L.host_hess_schur.argtypes = [P, P, P, P, ctypes.c_int]
    L.host_lno_atom.argtypes = [P, P, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, P]
    return L


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _schur(lib, A):
    m = A.shape[0]
    a = np.zeros((LD, LD))
    a[:m, :m] = A
    z = np.zeros((LD, LD))
    wr, wi = np.zeros(LD), np.zeros(LD)
    st = lib.host_hess_schur(_p(a), _p(z), _p(wr), _p(wi), m)
    return st, a[:m, :m].copy(), z[:m, :m].copy(), wr[:m] + 1j * wi[:m]


def _cases():
    rng = np.random.default_rng(20251203)
    out = []
    for m in range(1, 17):
        for t in range(6):
            out.append(rng.standard_normal((m, m)) * (10.0 ** rng.integers(-3, 3)))
    # cyclic shifts and their perturbations: the unshifted-QR fixed points that need ad hoc shifts
    for m in (3, 4, 7, 16):
        P = np.roll(np.eye(m), 1, axis=0)
        out.append(P)
        out.append(P + 1e-9 * rng.standard_normal((m, m)))
    # exactly repeated and clustered eigenvalues, rotations (pure pairs), a defective block
    for m in (4, 9, 13):
        Q, _ = np.linalg.qr(rng.standard_normal((m, m)))
        out.append(Q @ np.diag(np.repeat([1.0, -0.5, 0.25], m)[:m]) @ Q.T)
        out.append(Q)
    out.append(np.array([[1.0, 1.0], [0.0, 1.0]]))
    out.append(np.array([[0.0, -2.0], [3.0, 0.0]]))
    return out


def test_real_schur_form(lib):
    n_pairs = 0
    for A in _cases():
        m = A.shape[0]
        st, T, Z, w = _schur(lib, A)
        assert st == 0
        sc = max(1.0, np.abs(A).max())
        # orthogonal similarity: Z^T A Z = T, Z^T Z = I
        assert np.abs(Z.T @ Z - np.eye(m)).max() <= 1e-13 * m
        assert np.abs(Z.T @ A @ Z - T).max() <= 1e-13 * m * sc
        # quasi-triangular: nothing below the subdiagonal, no two consecutive subdiagonal entries,
        # and a nonzero subdiagonal entry only inside a complex pair's 2 x 2 block
        assert np.all(np.tril(T, -2) == 0.0)
        sub = np.diag(T, -1)
        assert not np.any((sub[:-1] != 0.0) & (sub[1:] != 0.0))
        for p in np.nonzero(sub)[0]:
            assert w[p].imag > 0 and w[p + 1].imag < 0 and w[p].real == w[p + 1].real
            n_pairs += 1
        # the same eigenvalues as LAPACK (as multisets)
        ref = np.linalg.eigvals(A)
        assert np.abs(np.sort_complex(np.round(w, 9)) - np.sort_complex(np.round(ref, 9))).max() <= 1e-7 * sc or \
            all(np.min(np.abs(ref - x)) <= 1e-6 * sc for x in w)
    assert n_pairs >= 50  # the cases exercise many complex-conjugate pairs


def _lambda_like(rng, m, pair_gap=None):
    """A nonsymmetric m x m matrix with eigenvalues spread over (-0.2, 1.2) and some complex pairs,
    and an SPD S_jj block."""
    V = rng.standard_normal((m, m))
    D = np.zeros((m, m))
    vals = np.sort(rng.uniform(-0.2, 1.2, m))[::-1]
    i = 0
    while i < m:
        if i + 1 < m and rng.random() < 0.4:
            a, b = vals[i], 0.05 + 0.2 * rng.random()
            D[i:i + 2, i:i + 2] = [[a, b], [-b, a]]
            i += 2
        else:
            D[i, i] = vals[i]
            i += 1
    lam = V @ D @ np.linalg.inv(V)
    x = rng.standard_normal((m, m)) * 0.1
    sjj = np.eye(m) + 0.5 * (x + x.T) * 0.3
    return lam, sjj


def _projector(U, sjj):
    # S-orthogonal projector onto span U: U (U^T S U)^{-1} U^T S
    return U @ np.linalg.solve(U.T @ sjj @ U, U.T @ sjj)


def _host_lno(lib, lam, sjj, th, kmin, kmax, fixed):
    m = lam.shape[0]
    a = np.zeros((LD, LD))
    a[:m, :m] = lam
    s = np.zeros((LD, LD))
    s[:m, :m] = sjj
    u = np.zeros(LD * LD)
    k = lib.host_lno_atom(_p(a), _p(s), m, th, kmin, kmax, fixed, _p(u))
    return k, u[: m * max(k, 0)].reshape(max(k, 0), m).T if k > 0 else np.zeros((m, 0))


def test_lno_atom_against_lapack(lib):
    rng = np.random.default_rng(7)
    seen = {"kept_pair": 0, "cut_pair": 0, "dropped_pair": 0}
    for trial in range(300):
        m = int(rng.integers(1, 17))
        lam, sjj = _lambda_like(rng, m)
        th = float(rng.uniform(-0.1, 1.1))
        kmin, kmax = 1, (-1 if trial % 3 else int(rng.integers(1, m + 1)))
        fixed = -1 if trial % 4 else int(rng.integers(0, m + 1))
        w, V = olno.sorted_eig(lam)
        k_ref = olno.select_rank(w, th, kmin, kmax, None if fixed < 0 else fixed)
        k, U = _host_lno(lib, lam, sjj, th, kmin, kmax, fixed)
        assert k == k_ref, (trial, m, k, k_ref)
        if k == 0:
            continue
        # classify what the cut did to a pair
        wi = w.imag
        kept = wi[:k] != 0
        if np.any(kept):
            seen["kept_pair"] += 1
        if k < m and np.any(wi[k:] != 0):
            seen["dropped_pair"] += 1
        raw = (min(fixed, m) if fixed >= 0 else int(np.clip(np.sum(w.real >= th), kmin, m if kmax < 0 else kmax)))
        if raw != k:
            seen["cut_pair"] += 1
        # S_jj-orthonormal basis of the same span as the oracle's
        assert np.abs(U.T @ sjj @ U - np.eye(k)).max() <= 1e-11
        Uo = olno.lowdin(olno.real_basis(w, V, k), sjj)
        assert np.abs(_projector(U, sjj) - _projector(Uo, sjj)).max() <= 1e-9
    assert min(seen.values()) >= 5, seen
