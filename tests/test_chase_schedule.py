"""Host model of the bulge-chasing kernel's schedule (csrc/k_tridiag.hip, sb2st_kernel).

The kernel runs the sweeps of the band-to-tridiagonal reduction in pairs (2p, 2p + 1) on one
wavefront and never loads the second sweep's windows: each is built in registers from the first
sweep's previous window (moved down and right by one row and column), the first column of the first
sweep's current window, and a zero last row.  This model replays that dataflow on a band array in
numpy, with the kernel's window masks, store modes and pair-start rule, and checks it against the
plain schedule in which every step loads and stores its own window: the reflectors, the diagonal and
the off-diagonal must agree bit for bit (both schedules run the same step arithmetic, so any
difference is a dataflow error: a stale entry, a missed store, a wrong shift).  It also checks the
chase's traffic model in bench.py against the loads and stores the model makes.  The step itself
is the Householder bulge-chasing step (Sec. II.C (iii)); the tridiagonal's eigenvalues are checked
against numpy's so that a broken step cannot pass as two equally broken schedules.
"""
import os
import sys

import numpy as np
import pytest

B = 32   # band width
LB = 80  # band array column stride (2B + 1 diagonals, padded)


def steps(n, s):
    return 0 if s > n - 3 else (n - 3 - s) // B + 1


class Band:
    """Lower band + bulge of a symmetric matrix: entry (r, c), r >= c, at column c, offset r - c."""

    def __init__(self, A):
        self.n = n = A.shape[0]
        self.a = np.zeros((n, LB))
        for c in range(n):
            for d in range(B + 1):
                if c + d < n:
                    self.a[c, d] = A[c + d, c]
        self.refl = {}
        self.loads = 0
        self.stores = 0

    def ld(self, r, c):
        if r >= self.n or c >= self.n:
            return 0.0
        assert 0 <= r - c < LB
        return self.a[c, r - c]

    def st(self, r, c, v):
        if r >= self.n or c >= self.n:
            return
        assert 0 <= r - c < LB
        self.a[c, r - c] = v


def geometry(n, s, j):
    r0 = s + 1 + j * B
    ln = min(B, n - r0)
    return r0, ln, max(0, min(B, n - r0 - ln))


def in_window(l, k, ln, nr):
    """Lane l (D rows 0..31, R rows 32..63), column k: an entry the step loads and stores."""
    return (l >= k and l < ln) if l < 32 else ((l - 32) < nr and k < ln)


def fetch(bd, s, j):
    n = bd.n
    r0, ln, nr = geometry(n, s, j)
    W = np.zeros((64, B))
    for l in range(64):
        for k in range(B):
            if in_window(l, k, ln, nr):
                W[l, k] = bd.ld(r0 + l, r0 + k)
                bd.loads += 1
    return W


def column(bd, s):
    return np.array([bd.ld(s + 1 + i, s) for i in range(32)])


def householder(x, m):
    """Reflector of x[:m] (x[0] the pivot): tau, v (v[0] = 1), beta."""
    sigma = float(np.sum(x[1:m] ** 2))
    alpha = x[0]
    if sigma == 0.0:
        return 0.0, np.eye(1, 32, 0)[0] * (m > 0), alpha
    beta = -np.copysign(np.sqrt(alpha * alpha + sigma), alpha)
    v = np.zeros(32)
    v[0] = 1.0
    v[1:m] = x[1:m] / (alpha - beta)
    return (beta - alpha) / beta, v, beta


def step(bd, W, x, s, j, slot):
    """Bulge step (s, j) on the window W (rows on lanes); the reflectors go to bd.refl."""
    n = bd.n
    r0, ln, nr = geometry(n, s, j)
    if j == 0:
        tau, v, beta = householder(np.where(np.arange(32) < ln, x, 0.0), ln)
        for i in range(32):
            bd.st(s + 1 + i, s, beta if i == 0 else 0.0)
        for i in range(ln):
            bd.refl[(s, i)] = tau if i == 0 else v[i]
        slot["tau"], slot["v"] = tau, v
    tau, v = slot["tau"], slot["v"].copy()
    D = np.array([[W[max(i, k), min(i, k)] for k in range(32)] for i in range(32)])
    W[:32] = D
    rows = np.arange(64)
    isrow = (rows < 32) & (rows < ln)
    isr = (rows >= 32) & (rows - 32 < nr)
    p = tau * (W @ v)
    vp = float(np.sum(np.where(isrow[:32], v * p[:32], 0.0)))
    w = np.where(isrow[:32], p[:32] - 0.5 * tau * vp * v, 0.0)
    for l in range(64):
        if l < 32:
            if isrow[l]:
                W[l] = W[l] - w[l] * v - v[l] * w
        elif isr[l]:
            W[l] = W[l] - p[l] * v
    if nr >= 2:
        tau1, v1, beta = householder(np.where(isr, W[:, 0], 0.0)[32:], nr)
        W[32:, 0] = 0.0
        W[32, 0] = beta
        for i in range(nr):
            bd.refl[(s, (j + 1) * B + i)] = tau1 if i == 0 else v1[i]
        slot["tau"], slot["v"] = tau1, v1
        wv = tau1 * (v1 @ W[32:, 1:])
        W[32:, 1:] -= np.outer(v1, wv)


ALL, DIAG, COL0_TAIL, ALL_BUT_COL0 = range(4)


def store(bd, W, s, j, mode=ALL):
    n = bd.n
    r0, ln, nr = geometry(n, s, j)
    for l in range(64):
        for k in range(B):
            if not in_window(l, k, ln, nr):
                continue
            if mode == DIAG and not (l == 0 and k == 0):
                continue
            if mode == COL0_TAIL and not (k == 0 and l >= 33):
                continue
            if mode == ALL_BUT_COL0 and not (k >= 1 or l >= 33):
                continue
            if r0 + l < n and r0 + k < n:
                bd.st(r0 + l, r0 + k, W[l, k])
                bd.stores += 1


def run_plain(A):
    """One sweep per step, every step loading and storing its window."""
    bd = Band(A)
    n = bd.n
    slots = {}
    for t in range(0, 2 * (n - 3) + 1):
        for s in range(min(t // 2, n - 3), -1, -1):
            j = t - 2 * s
            if j >= steps(n, s):
                break
            W = fetch(bd, s, j)
            step(bd, W, column(bd, s) if j == 0 else None, s, j, slots.setdefault(s, {}))
            store(bd, W, s, j)
    return bd


def pair_last(n, p):
    s = 2 * p
    return steps(n, s + 1) if s + 1 <= n - 3 else steps(n, s) - 1


def pair_starts(n, nw):
    T = []
    for p in range((n - 1) // 2 if n >= 3 else 0):
        t = 0 if p == 0 else T[p - 1] + 3
        if p >= nw:
            t = max(t, T[p - nw] + pair_last(n, p - nw) + 1)
        T.append(t)
    return T


def run_pairs(A, nw, forward):
    """The kernel's schedule: pairs of sweeps, the second sweep's windows built from the first's."""
    bd = Band(A)
    n = bd.n
    T = pair_starts(n, nw)
    if not T:
        return bd
    P, slots = {}, {}
    for t in range(max(T[p] + pair_last(n, p) for p in range(len(T))) + 1):
        order = range(len(T)) if forward else range(len(T) - 1, -1, -1)
        for p in order:
            tau = t - T[p]
            if tau < 0 or tau > pair_last(n, p):
                continue
            s = 2 * p
            solo = s + 1 > n - 3
            J0 = steps(n, s)
            J1 = 0 if solo else steps(n, s + 1)
            C = None
            if tau < J0:
                C = fetch(bd, s, tau)
                step(bd, C, column(bd, s) if tau == 0 else None, s, tau, slots.setdefault(s, {}))
                mode = ALL if solo else DIAG if tau == 0 else ALL_BUT_COL0 if (tau == J0 - 1 and J1 <= tau) \
                    else COL0_TAIL
                store(bd, C, s, tau, mode)
            if tau >= 1 and tau - 1 < J1:
                r0c = s + 1 + tau * B
                if C is not None:
                    c0 = C[:, 0]
                else:
                    c0 = np.zeros(64)
                    if r0c <= n - 1:
                        for l in range(B + 1):
                            c0[l] = bd.ld(r0c + l, r0c)
                            bd.loads += r0c + l < n
                S = np.zeros((64, B))
                S[:63, :B - 1] = P[p][1:, 1:]
                S[B - 1:, B - 1] = c0[:64 - (B - 1)]
                step(bd, S, P[p][1:33, 0], s + 1, tau - 1, slots.setdefault(s + 1, {}))
                store(bd, S, s + 1, tau - 1)
            if C is not None:
                P[p] = C
    return bd


def _bench_ns():
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    ns = {"__name__": "bench_model", "__file__": os.path.join(root, "bench.py")}
    argv = sys.argv
    try:
        sys.argv = ["bench.py"]
        with open(os.path.join(root, "bench.py")) as f:
            exec(compile(f.read(), "bench.py", "exec"), ns)
    finally:
        sys.argv = argv
    return ns


def _matrix(n, seed):
    M = np.random.default_rng(seed).standard_normal((n, n))
    return np.tril(np.triu(M + M.T, -B), B)


@pytest.mark.parametrize("n", [3, 4, 5, 34, 35, 66, 67, 97, 131])
@pytest.mark.parametrize("nw", [1, 2, 4])
def test_pairs_match_plain_schedule(n, nw):
    A = _matrix(n, 100 * n + nw)
    a = run_plain(A)
    for forward in (False, True):
        b = run_pairs(A, nw, forward)
        assert np.array_equal(a.a[:, 0], b.a[:, 0]), "diagonal"
        assert np.array_equal(a.a[:n - 1, 1], b.a[:n - 1, 1]), "off-diagonal"
        assert a.refl.keys() == b.refl.keys()
        assert all(a.refl[k] == b.refl[k] for k in a.refl), "reflectors"
    # the step is a similarity transform: T has A's eigenvalues
    d, e = a.a[:, 0], a.a[:n - 1, 1]
    T = np.diag(d) + np.diag(e, -1) + np.diag(e, 1)
    ev = np.linalg.eigvalsh(A)
    assert np.max(np.abs(np.linalg.eigvalsh(T) - ev)) <= 1e-12 * max(1.0, np.max(np.abs(ev))) * n


def test_pair_starts_leave_columns_disjoint():
    """Pairs three pair times apart: at every pair time, steps of different pairs touch disjoint
    columns of the band array (step 0 also writes column s), and a wave runs one pair at a time."""
    for n in (35, 97, 300, 693):
        for nw in (1, 2, 8):
            T = pair_starts(n, nw)
            owner = {}
            for p, t0 in enumerate(T):
                s = 2 * p
                assert p < nw or t0 > T[p - nw] + pair_last(n, p - nw), "a wave runs one pair at a time"
                for tau in range(pair_last(n, p) + 1):
                    spans = []
                    if tau < steps(n, s):
                        spans.append((s, tau))
                    if s + 1 <= n - 3 and 1 <= tau and tau - 1 < steps(n, s + 1):
                        spans.append((s + 1, tau - 1))
                    for (ss, j) in spans:
                        r0, ln, _ = geometry(n, ss, j)
                        for c in list(range(r0, r0 + ln)) + ([ss] if j == 0 else []):
                            key = (t0 + tau, c)
                            assert owner.get(key, p) == p, (n, nw, key)
                            owner[key] = p


@pytest.mark.parametrize("n", [5, 35, 66, 67, 131])
def test_bench_chase_traffic_model(n):
    """bench.py's window traffic of the chase equals the model's loads and stores, plus one
    reflector entry per window row (the formula's len doubles per step)."""
    ns = _bench_ns()
    b = run_pairs(_matrix(n, n), 2, False)
    refl = sum(geometry(n, s, j)[1] for s in range(n - 2) for j in range(steps(n, s)))
    assert ns["sb2st_design_bytes"](np.array([n])) == 8.0 * (b.loads + b.stores + refl)
