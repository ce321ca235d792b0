"""Seeded synthetic tight-binding inputs for DC-LNO density builds.

This module is the only code that the CPU oracle and the GPU path share, and it holds
none of the method's arithmetic: it places atoms on a lattice, draws random Hamiltonian
and overlap blocks on a distance-cutoff pattern, and states the run parameters (cluster
radius, temperature, electron count, LNO rank rule).  Everything the method computes
(clusters, regions, LNOs, eigenpairs, chemical potential, density rows) lives elsewhere.

Matrix layout (both sides read it): variable-size block-sparse rows (BSR) with one block
per atom pair, images folded onto the same pair (a Gamma-point supercell).  Row i holds
the blocks (i, j) for every j in the structural pattern of i, j ascending, the diagonal
block included.  Block (i, j) is an M_i x M_j row-major float64 array starting at element
``blk_off[b]`` of the flat value array.  H, S and any density matrix share the pattern.

Units: lengths are in units of the lattice's nearest-neighbour distance unless a caller
passes an explicit lattice constant, energies in Hartree.
"""
from __future__ import annotations

import itertools
import math
import os

import numpy as np
from numpy.random import Generator, PCG64

SEED_BASE = 1809_05637 * 10

_BASIS = {
    "sc": np.array([[0.0, 0.0, 0.0]]),
    "bcc": np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]]),
    "fcc": np.array([[0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0]]),
}
_BASIS["diamond"] = np.vstack([_BASIS["fcc"], _BASIS["fcc"] + 0.25])

# nearest-neighbour distance in units of the conventional lattice constant
NN_DISTANCE = {"sc": 1.0, "bcc": math.sqrt(3.0) / 2.0, "fcc": math.sqrt(0.5), "diamond": math.sqrt(3.0) / 4.0}

# first neighbour shells in units of the nearest-neighbour distance (ideal lattices)
SHELLS = {
    "diamond": [1.0, math.sqrt(8 / 3), math.sqrt(11 / 3), math.sqrt(16 / 3), math.sqrt(19 / 3),
                math.sqrt(8.0), 3.0, math.sqrt(32 / 3), math.sqrt(35 / 3), math.sqrt(40 / 3)],
    "fcc": [1.0, math.sqrt(2.0), math.sqrt(3.0), 2.0, math.sqrt(5.0), math.sqrt(6.0), math.sqrt(7.0)],
    "sc": [1.0, math.sqrt(2.0), math.sqrt(3.0), 2.0, math.sqrt(5.0), math.sqrt(6.0)],
}


def lattice(kind: str, cells, a: float | None = None):
    """Atoms of ``cells`` = (nx, ny, nz) conventional cubic cells of a lattice.

    Returns (pos (N,3), cell (3,3), sublattice (N,)).  Atom order: cell index x, then y,
    then z, then basis atom.  ``a`` defaults to the value that makes the nearest-neighbour
    distance 1.  For diamond the sublattice is 0 for the fcc sites and 1 for the shifted ones.
    """
    basis = _BASIS[kind]
    if a is None:
        a = 1.0 / NN_DISTANCE[kind]
    nx, ny, nz = cells
    grid = np.array(list(itertools.product(range(nx), range(ny), range(nz))), dtype=np.float64)
    pos = (grid[:, None, :] + basis[None, :, :]).reshape(-1, 3) * a
    sub = np.tile(np.arange(len(basis)) >= (len(basis) // 2 if kind == "diamond" else len(basis)),
                  len(grid)).astype(np.int32)
    cell = np.diag([nx * a, ny * a, nz * a]).astype(np.float64)
    return pos, cell, sub


def bonds(pos, cell, periodic, rcut, tol=1e-9):
    """All bonds (i, j, R) with |pos_j + R.cell - pos_i| <= rcut (+tol).

    Canonical order: i ascending, j >= i ascending, then the integer image vector R in
    lexicographic order; a bond of an atom with its own image keeps only R > 0
    (lexicographically), so every bond appears once.  Returns (i, j, R (B,3), r (B,)).
    """
    from scipy.spatial import cKDTree

    pos = np.asarray(pos, dtype=np.float64)
    lengths = np.diag(cell)
    ranges = []
    for ax in range(3):
        if periodic[ax]:
            m = int(math.ceil((rcut + tol) / lengths[ax])) + 1
            ranges.append(range(-m, m + 1))
        else:
            ranges.append(range(0, 1))
    tree = cKDTree(pos)
    out_i, out_j, out_R, out_r = [], [], [], []
    for R in itertools.product(*ranges):
        R = np.array(R)
        shift = R * lengths
        other = cKDTree(pos + shift)
        sdm = tree.sparse_distance_matrix(other, rcut + tol, output_type="ndarray")
        if len(sdm) == 0:
            continue
        i = sdm["i"].astype(np.int64)
        j = sdm["j"].astype(np.int64)
        r = sdm["v"]
        Rlex = tuple(R)
        keep = (i < j) | ((i == j) & (Rlex > (0, 0, 0)))
        keep &= r > 1e-12
        i, j, r = i[keep], j[keep], r[keep]
        out_i.append(i)
        out_j.append(j)
        out_R.append(np.repeat(R[None, :], len(i), axis=0))
        out_r.append(r)
    i = np.concatenate(out_i)
    j = np.concatenate(out_j)
    R = np.concatenate(out_R).astype(np.int64)
    r = np.concatenate(out_r)
    order = np.lexsort((R[:, 2], R[:, 1], R[:, 0], j, i))
    return i[order], j[order], R[order], r[order]


def bsr_pattern(n_atoms, bi, bj):
    """Row pointers and sorted columns of the pattern {(i,i)} U {(i,j),(j,i) for bonds}."""
    keys = np.concatenate([np.arange(n_atoms, dtype=np.int64) * (n_atoms + 1),
                           bi * n_atoms + bj, bj * n_atoms + bi])
    keys = np.unique(keys)
    rows = keys // n_atoms
    cols = keys % n_atoms
    row_ptr = np.zeros(n_atoms + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return row_ptr.astype(np.int32), cols.astype(np.int32), keys


def _block_offsets(n_orb, row_ptr, col):
    rows = np.repeat(np.arange(len(n_orb)), np.diff(row_ptr))
    sizes = n_orb[rows].astype(np.int64) * n_orb[col].astype(np.int64)
    off = np.zeros(len(col) + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    return off


def assemble(n_atoms, n_orb, bi, bj, br, onsite_h, h_scale, s_scale, rng):
    """Draw one Gaussian block per bond for H, then one per bond for S, and fold them.

    H_ij += h_scale(r) * B and H_ji += (h_scale(r) * B)^T for every bond; S likewise with
    its own blocks; H_ii = diag(onsite_h[i]), S_ii = I.  Returns the BSR arrays.
    """
    row_ptr, col, keys = bsr_pattern(n_atoms, bi, bj)
    blk_off = _block_offsets(n_orb, row_ptr, col)
    mmax = int(n_orb.max())
    nnzb = len(col)
    key_ij = bi * n_atoms + bj
    key_ji = bj * n_atoms + bi
    idx_ij = np.searchsorted(keys, key_ij)
    idx_ji = np.searchsorted(keys, key_ji)
    mi = n_orb[bi]
    mj = n_orb[bj]

    def draw(nb):
        # one M_i x M_j standard-normal block per bond, bonds in canonical order, each
        # block filled in row-major order
        sizes = (mi * mj).astype(np.int64)
        flat = rng.standard_normal(int(sizes.sum()))
        blocks = np.zeros((nb, mmax, mmax))
        if np.all(mi == mmax) and np.all(mj == mmax):
            blocks[:] = flat.reshape(nb, mmax, mmax)
        else:
            off = np.concatenate([[0], np.cumsum(sizes)])
            for b in range(nb):
                blocks[b, : mi[b], : mj[b]] = flat[off[b]: off[b + 1]].reshape(mi[b], mj[b])
        return blocks

    nb = len(bi)
    out = []
    for scale, diag_kind in ((h_scale, "h"), (s_scale, "s")):
        blocks = draw(nb) * scale[:, None, None]
        dense = np.zeros((nnzb, mmax, mmax))
        np.add.at(dense, idx_ij, blocks)
        np.add.at(dense, idx_ji, np.transpose(blocks, (0, 2, 1)))
        diag_idx = np.searchsorted(keys, np.arange(n_atoms, dtype=np.int64) * (n_atoms + 1))
        for a in range(n_atoms):
            m = n_orb[a]
            if diag_kind == "h":
                dense[diag_idx[a], :m, :m] += np.diag(onsite_h[a][:m])
            else:
                dense[diag_idx[a], :m, :m] += np.eye(m)
        flat = np.empty(int(blk_off[-1]))
        rows = np.repeat(np.arange(n_atoms), np.diff(row_ptr))
        if np.all(n_orb == mmax):
            flat[:] = dense.reshape(-1)
        else:
            for b in range(nnzb):
                m1, m2 = n_orb[rows[b]], n_orb[col[b]]
                flat[blk_off[b]: blk_off[b + 1]] = dense[b, :m1, :m2].reshape(-1)
        out.append(flat)
    return row_ptr, col, blk_off[:-1].copy(), out[0], out[1]


def bsr_to_scipy(sysd, values):
    """Assemble a BSR value array into a scipy CSR matrix (test and generator helper)."""
    import scipy.sparse as sp

    n_orb = sysd["n_orb"]
    offs = np.zeros(len(n_orb) + 1, dtype=np.int64)
    offs[1:] = np.cumsum(n_orb)
    rows_i, cols_i, vals = [], [], []
    row_ptr, col, blk_off = sysd["row_ptr"], sysd["col"], sysd["blk_off"]
    for i in range(len(n_orb)):
        for b in range(row_ptr[i], row_ptr[i + 1]):
            j = col[b]
            mi, mj = n_orb[i], n_orb[j]
            blk = values[blk_off[b]: blk_off[b] + mi * mj].reshape(mi, mj)
            r, c = np.meshgrid(np.arange(mi) + offs[i], np.arange(mj) + offs[j], indexing="ij")
            rows_i.append(r.ravel())
            cols_i.append(c.ravel())
            vals.append(blk.ravel())
    n = int(offs[-1])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows_i), np.concatenate(cols_i))), shape=(n, n))


def _min_eig_sparse(S):
    import scipy.sparse.linalg as sla

    if S.shape[0] <= 3000:
        return float(np.linalg.eigvalsh(S.toarray())[0])
    val = sla.eigsh(S, k=1, which="SA", tol=1e-8, maxiter=20000, return_eigenvectors=False)
    return float(val[0])


def make_system(kind, cells, periodic, n_orb_per_atom, onsite, t0, lam_h, hop_cut, seed,
                s_amp=0.05, lam_s=0.8, vacancies=0, min_s_eig=0.2, a=None):
    """Build one synthetic system.

    kind/cells/periodic: lattice; n_orb_per_atom: orbitals per atom, an int or a sequence
    tiled over the atoms; onsite: callable (rng, sublattice (N,), M) -> (N, M) onsite energies
    (M the largest count; atom i uses its first M_i); t0, lam_h: hopping amplitude and
    decay length (blocks scaled by t0*exp(-r/lam_h)); hop_cut: bond cutoff; s_amp, lam_s:
    overlap blocks scaled by s_amp*exp(-r/lam_s) on the same bonds; vacancies: number of
    sites removed, drawn from a second stream (seed + 1).  If the smallest eigenvalue of S
    is below ``min_s_eig`` the off-site overlap amplitude is halved until it is not; the
    factor used is recorded.
    """
    pos, cell, sub = lattice(kind, cells, a)
    if vacancies:
        vrng = Generator(PCG64(seed + 1))
        drop = vrng.choice(len(pos), size=vacancies, replace=False)
        keep = np.ones(len(pos), dtype=bool)
        keep[drop] = False
        pos, sub = pos[keep], sub[keep]
    n_atoms = len(pos)
    if np.ndim(n_orb_per_atom) == 0:
        n_orb = np.full(n_atoms, n_orb_per_atom, dtype=np.int32)
    else:
        n_orb = np.resize(np.asarray(n_orb_per_atom, dtype=np.int32), n_atoms)
    bi, bj, bR, br = bonds(pos, cell, periodic, hop_cut)
    factor = 1.0
    while True:
        rng = Generator(PCG64(seed))
        eps = onsite(rng, sub, int(n_orb.max()))
        h_scale = t0 * np.exp(-br / lam_h)
        s_scale = factor * s_amp * np.exp(-br / lam_s)
        row_ptr, col, blk_off, H, S = assemble(n_atoms, n_orb, bi, bj, br, eps, h_scale, s_scale, rng)
        sysd = dict(n_atoms=n_atoms, pos=pos, cell=cell, periodic=np.asarray(periodic, dtype=np.int32),
                    n_orb=n_orb, row_ptr=row_ptr, col=col, blk_off=blk_off, H=H, S=S, sublattice=sub)
        smin = _min_eig_sparse(bsr_to_scipy(sysd, S))
        if smin >= min_s_eig:
            break
        factor *= 0.5
    sysd["s_factor"] = factor
    sysd["s_min_eig"] = smin
    sysd["n_bonds"] = len(bi)
    return sysd


def _gap_at_half_filling(sysd):
    import scipy.linalg as sl

    H = bsr_to_scipy(sysd, sysd["H"]).toarray()
    S = bsr_to_scipy(sysd, sysd["S"]).toarray()
    e = sl.eigh(H, S, eigvals_only=True)
    n = len(e)
    return float(e[n // 2] - e[n // 2 - 1])


def _onsite_gauss(sigma):
    def f(rng, sub, m):
        return rng.normal(0.0, sigma, size=(len(sub), m))
    return f


def _onsite_sublattice(value):
    def f(rng, sub, m):
        return np.where(sub[:, None] == 0, value, -value) * np.ones((1, m))
    return f


def _onsite_split(value):
    """+-value per orbital half: on sublattice 0 the first half of the orbitals sits at
    +value and the second half at -value; sublattice 1 has the opposite signs.  Every atom
    then has M/2 orbitals below and M/2 above the gap."""
    def f(rng, sub, m):
        half = np.where(np.arange(m) < m // 2, 1.0, -1.0)[None, :]
        sign = np.where(sub[:, None] == 0, 1.0, -1.0)
        return value * sign * half
    return f


def _onsite_zero(rng, sub, m):
    return np.zeros((len(sub), m))


_T0_LADDER = (1.0, 0.5, 0.2, 0.1, 0.05, 0.02, 0.01)


def diamond_t0(seed, m=8, lam_h=1.2, min_gap=0.2):
    """Largest hopping amplitude from a fixed ladder whose 2x2x2-cell periodic replica
    (64 atoms) keeps a gap >= min_gap Ha at half filling.  Returns (t0, gap)."""
    for t0 in _T0_LADDER:
        rep = make_system("diamond", (2, 2, 2), (1, 1, 1), m, _onsite_split(0.15), t0, lam_h,
                          SHELLS["diamond"][1] + 1e-6, seed)
        gap = _gap_at_half_filling(rep)
        if gap >= min_gap:
            return t0, gap
    return _T0_LADDER[-1], gap


def _params(sysd, name, r_L, kT, lno, lambda_th=0.1, k_min=1, k_max=-1, fixed_k=-1, kappa=0.3):
    n_basis = int(sysd["n_orb"].sum())
    sysd.update(name=name, r_L=float(r_L), kappa=float(kappa), kT=float(kT), spin_g=2,
                n_electrons=float(n_basis), n_basis=n_basis, lno=bool(lno), lambda_th=float(lambda_th),
                k_min=int(k_min), k_max=int(k_max), fixed_k=int(fixed_k))
    return sysd


def config(k: int, seed: int | None = None):
    """The benchmark systems by index.

    0: simple cubic 4x4x4 torus, 64 atoms x 4 orbitals, plain DC, r_L = 2.5, kT = 0.01.
    1: gapped diamond 5x5x5 cells (1000 atoms x 8 orbitals), onsite +-0.15 (the sublattice
       sign flips which half of the orbitals is low), hoppings to
       the 2nd shell, t0 from the gap ladder, r_L = 3.0 (7 shells), 4 LNOs per long atom,
       kT = 0.005.
    2: metallic fcc slab 10x10x10 cells, periodic in x and y, 80 vacancies (3920 atoms x 9
       orbitals), onsite 0, hoppings to the 3rd shell, r_L = sqrt(5) (5 shells),
       LNO rank = clamp(#{lambda >= 1e-3}, 2, 6), kT = 0.01.
    3: the config-2 system (the reduced-precision form runs on it).
    """
    if seed is None:
        seed = SEED_BASE + k
    if k == 0:
        s = make_system("sc", (4, 4, 4), (1, 1, 1), 4, _onsite_gauss(0.1), 1.0, 0.8, 2.5, seed)
        return _params(s, "sc64_plain", 2.5, 0.01, lno=False)
    if k == 1:
        t0, gap = diamond_t0(seed)
        s = make_system("diamond", (5, 5, 5), (1, 1, 1), 8, _onsite_split(0.15), t0, 1.2,
                        SHELLS["diamond"][1] + 1e-6, seed)
        s["t0"], s["replica_gap"] = t0, gap
        return _params(s, "diamond1000_gapped", 3.0, 0.005, lno=True, fixed_k=4)
    if k in (2, 3):
        s = make_system("fcc", (10, 10, 10), (1, 1, 0), 9, _onsite_zero, 1.0, 1.0,
                        SHELLS["fcc"][2] + 1e-6, SEED_BASE + 2 if seed is None else seed, vacancies=80)
        return _params(s, "fcc3920_metal_slab", math.sqrt(5.0), 0.01, lno=True, lambda_th=1e-3,
                       k_min=2, k_max=6)
    raise ValueError(f"unknown config {k}")


def small(name: str, seed: int = SEED_BASE + 100):
    """Reduced systems with the same recipes, for parity runs the oracle finishes quickly.

    'sc27':   simple cubic 3x3x3 torus, 4 orbitals, plain DC (r_L = 1.5).
    'dia216': diamond 3x3x3 cells (216 atoms), config-1 recipe, r_L = 2.52 (5 shells).
    'fcc_slab': fcc 4x4x3 cells periodic in x,y, 4 vacancies, config-2 recipe.
    'fcc256':  bulk fcc 4x4x4 cells, periodic, config-2 recipe without vacancies.
    'mixed27', 'mixed64': simple cubic with 1..16 orbitals per atom (plain DC; DC-LNO).
    'isolated': no bonds, one-atom clusters of 1..16 orbitals.
    'maxdim':  simple cubic 5x5x5, 16 orbitals, 57-atom clusters (dimension 912).
    'maxdim952': fcc 3x3x3 cells, orbital pattern 16,16,16,16,4, r_L = 2.4: clusters of
               dimension 880..952 (past 947 the tridiagonal solver's LDS exceeds 64 KB).
    'chain_gap' / 'chain_metal': 1D rings for truncation-behaviour checks.
    """
    if name == "sc27":
        s = make_system("sc", (3, 3, 3), (1, 1, 1), 4, _onsite_gauss(0.1), 1.0, 0.8, 1.5, seed)
        return _params(s, name, 1.5, 0.01, lno=False)
    if name == "sc64_whole":
        s = make_system("sc", (4, 4, 4), (1, 1, 1), 4, _onsite_gauss(0.1), 1.0, 0.8, 2.5, SEED_BASE)
        return _params(s, name, math.sqrt(12.0), 0.01, lno=False)
    if name == "dia216":
        t0, gap = diamond_t0(SEED_BASE + 1)
        s = make_system("diamond", (3, 3, 3), (1, 1, 1), 8, _onsite_split(0.15), t0, 1.2,
                        SHELLS["diamond"][1] + 1e-6, seed)
        s["t0"] = t0
        return _params(s, name, SHELLS["diamond"][4], 0.005, lno=True, fixed_k=4)
    if name == "fcc_slab":
        s = make_system("fcc", (4, 4, 3), (1, 1, 0), 9, _onsite_zero, 1.0, 1.0, SHELLS["fcc"][2] + 1e-6,
                        seed, vacancies=4)
        return _params(s, name, math.sqrt(5.0), 0.01, lno=True, lambda_th=1e-3, k_min=2, k_max=6)
    if name == "mixed27":
        # ragged blocks: 1, 4, 9, 16 and 5 orbitals per atom in turn (16 is the compiled limit)
        s = make_system("sc", (3, 3, 3), (1, 1, 1), [1, 4, 9, 16, 5], _onsite_gauss(0.1), 1.0, 0.8, 1.5, seed)
        return _params(s, name, 1.5, 0.01, lno=False)
    if name == "mixed64":
        # ragged blocks with a long region (DC-LNO, occupation rule, ranks 1..M_j)
        s = make_system("sc", (4, 4, 4), (1, 1, 1), [4, 9, 16, 6, 1], _onsite_gauss(0.1), 1.0, 0.8, 1.5, seed)
        return _params(s, name, 2.0, 0.01, lno=True, lambda_th=0.1, k_min=1, k_max=-1)
    if name == "isolated":
        # no bonds: every cluster is its own atom, of 1 to 16 orbitals (dimensions below one
        # band panel, the smallest tridiagonal problems)
        s = make_system("sc", (2, 2, 4), (1, 1, 1), list(range(1, 17)), _onsite_gauss(0.3), 1.0, 0.8, 0.5, seed)
        return _params(s, name, 0.5, 0.01, lno=False)
    if name == "maxdim":
        # 57-atom clusters of 16 orbitals: dimension 912, close to the compiled limit of 960
        s = make_system("sc", (5, 5, 5), (1, 1, 1), 16, _onsite_gauss(0.1), 1.0, 0.8, 1.5, seed)
        return _params(s, name, math.sqrt(5.0), 0.01, lno=False)
    if name == "maxdim952":
        s = make_system("fcc", (3, 3, 3), (1, 1, 1), [16, 16, 16, 16, 4], _onsite_gauss(0.1), 1.0, 0.8, 1.5, seed)
        return _params(s, name, 2.4, 0.01, lno=False)
    if name == "fcc256":
        # bulk fcc 4x4x4 cells, periodic, config-2 recipe (no vacancies): the metal of the
        # error-versus-cluster-radius sweep (box half-width 2.83 d_NN > the largest swept r_L)
        s = make_system("fcc", (4, 4, 4), (1, 1, 1), 9, _onsite_zero, 1.0, 1.0, SHELLS["fcc"][2] + 1e-6, seed)
        return _params(s, name, math.sqrt(5.0), 0.01, lno=True, lambda_th=1e-3, k_min=2, k_max=6)
    raise ValueError(f"unknown small system {name}")


def ring(n_sites, eps=0.0, t=1.0, kT=0.05, r_L=None, dimer=0.0):
    """1D ring with one s orbital per site, S = I, onsite eps (+-dimer alternating), hopping t.

    Lattice spacing 1, periodic.  The cluster radius defaults to the whole ring."""
    pos = np.zeros((n_sites, 3))
    pos[:, 0] = np.arange(n_sites)
    cell = np.diag([float(n_sites), 1e3, 1e3])
    n_orb = np.ones(n_sites, dtype=np.int32)
    bi = np.arange(n_sites, dtype=np.int64)
    bj = (bi + 1) % n_sites
    lo = np.minimum(bi, bj)
    hi = np.maximum(bi, bj)
    row_ptr, col, keys = bsr_pattern(n_sites, lo, hi)
    blk_off = np.arange(len(col), dtype=np.int64)
    H = np.zeros(len(col))
    S = np.zeros(len(col))
    rows = np.repeat(np.arange(n_sites), np.diff(row_ptr))
    diag = rows == col
    H[diag] = eps + dimer * np.where(rows[diag] % 2 == 0, 1.0, -1.0)
    H[~diag] = t
    S[diag] = 1.0
    sysd = dict(n_atoms=n_sites, pos=pos, cell=cell, periodic=np.array([1, 0, 0], dtype=np.int32),
                n_orb=n_orb, row_ptr=row_ptr, col=col, blk_off=blk_off, H=H, S=S,
                sublattice=np.zeros(n_sites, dtype=np.int32))
    return _params(sysd, "ring", n_sites / 2.0 if r_L is None else r_L, kT, lno=False)


def cache_dir():
    d = os.environ.get("LDC_CACHE", "/tmp/ldc_synth_cache")
    os.makedirs(d, exist_ok=True)
    return d


def load_config(k: int):
    """``config(k)`` with an on-disk cache (npz) keyed by the config index."""
    path = os.path.join(cache_dir(), f"config{k}_v1.npz")
    if os.path.exists(path):
        with np.load(path, allow_pickle=False) as z:
            d = {key: z[key] for key in z.files}
        for key, val in list(d.items()):
            if val.ndim == 0:
                d[key] = val.item()
        return d
    d = config(k)
    np.savez(path, **{key: np.asarray(val) for key, val in d.items()})
    return d
