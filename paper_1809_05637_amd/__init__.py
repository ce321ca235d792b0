"""MI355X (gfx950) DC-LNO density builds: thin ctypes binding of libldc.so.

The library is the product: every step of a density build (LNOs, cluster gather,
Cholesky, standard form, tridiagonalization, divide-and-conquer, chemical potential,
density rows) runs in its HIP kernels.  This module only marshals arguments; it passes
raw device pointers (torch tensors supply device memory and the stream).  It fails
loudly when the library is missing -- there is no CPU fallback.

Entry points mirror include/ldc.h: Plan.lno (ldc_lno), Plan.solve (ldc_solve),
Plan.density (ldc_density), Plan.build (ldc_build: the three in one call, optionally replayed
from a HIP graph), Plan.tune (ldc_tune), Plan.density_at (ldc_density_at), Plan.energy_density
(ldc_energy_density) and the rest of the header.  Device arguments are checked (float64,
contiguous, on the plan's GPU, of the pattern's length) before the call.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = ["Plan", "LdcError", "library_path", "load", "STATUS"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

STATUS = {0: "LDC_OK", 1: "LDC_ERR_ARG", 2: "LDC_ERR_NOT_SPD", 3: "LDC_ERR_EIG_NOCONV", 4: "LDC_ERR_MU_BRACKET",
          5: "LDC_ERR_RANK", 6: "LDC_ERR_OOM", 7: "LDC_ERR_DEVICE", 8: "LDC_ERR_STATE", 9: "LDC_ERR_LIMIT"}

NUM_STAGES = 11

c_int, c_double, c_void_p, c_size_t = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t
P_int = ctypes.POINTER(ctypes.c_int)
P_double = ctypes.POINTER(ctypes.c_double)


class Options(ctypes.Structure):
    _fields_ = [("r_L", c_double), ("kappa", c_double), ("dist_tol", c_double), ("shell_tol", c_double),
                ("spin_g", c_int), ("workgroups", c_int), ("prec", c_int), ("batched", c_int), ("use_graph", c_int),
                ("tune_cache", ctypes.c_char_p)]


class RankRule(ctypes.Structure):
    _fields_ = [("lambda_th", c_double), ("k_min", c_int), ("k_max", c_int), ("fixed_rank", P_int)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n_atoms", c_int), ("n_basis", c_int), ("nnzb", c_int), ("max_members", c_int),
                ("max_dim_pao", c_int), ("lno_mode", c_int), ("device_bytes", c_size_t), ("blk_total", ctypes.c_longlong),
                ("n_buckets", c_int), ("tuned", c_int), ("graph_captures", c_int), ("graph_replays", c_int)]


PREC = {"fp64": 0, "mixed_fp32": 1}
TUNED_STAGES = ("gather", "potrf", "sygst", "sy2sb", "sb2st", "q2x", "stedc", "density")


class LdcError(RuntimeError):
    def __init__(self, status, msg, where=-1):
        self.status = status
        self.name = STATUS.get(status, str(status))
        self.where = where
        super().__init__(f"{self.name}: {msg} (cluster/atom {where})")


def library_path():
    return os.path.join(_HERE, "libldc.so")


def load():
    """Load libldc.so (built in-tree by __graft_entry__.build()); raises if it is absent."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(path)
    sig = {
        "ldc_plan_create": (c_int, [ctypes.POINTER(c_void_p), c_int, P_double, P_double, P_int, P_int, c_int, P_int,
                                    P_int, ctypes.POINTER(Options), c_void_p]),
        "ldc_plan_destroy": (c_int, [c_void_p]),
        "ldc_plan_set_stream": (c_int, [c_void_p, c_void_p]),
        "ldc_plan_query": (c_int, [c_void_p, ctypes.POINTER(PlanInfo)]),
        "ldc_plan_cluster": (c_int, [c_void_p, c_int, P_int, P_int, P_int, P_int]),
        "ldc_regions": (c_int, [c_int, P_double, P_double, P_int, P_int, c_int, P_int, P_int,
                                ctypes.POINTER(Options), c_int, P_int, P_int, P_int]),
        "ldc_plan_buckets": (c_int, [c_void_p, P_int, P_int, P_int, P_int]),
        "ldc_lno": (c_int, [c_void_p, c_void_p, c_void_p, ctypes.POINTER(RankRule), P_int]),
        "ldc_build": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, ctypes.POINTER(RankRule), c_double, c_double,
                              c_void_p, P_double, P_double, P_double]),
        "ldc_tune": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, ctypes.POINTER(RankRule), c_double, c_double,
                             c_void_p, P_double]),
        "ldc_reference_populations": (c_int, [c_void_p, c_double, c_void_p]),
        "ldc_solve": (c_int, [c_void_p, c_void_p, c_void_p]),
        "ldc_density": (c_int, [c_void_p, c_double, c_double, c_void_p, P_double, P_double, P_double]),
        "ldc_density_at": (c_int, [c_void_p, c_double, c_double, c_void_p, P_double, P_double]),
        "ldc_density_noalloc": (c_int, [c_void_p, c_double, c_double, c_void_p, c_void_p]),
        "ldc_energy_density": (c_int, [c_void_p, c_void_p, P_double]),
        "ldc_window_density": (c_int, [c_void_p, c_double, c_double, c_double, c_void_p, P_double]),
        "ldc_mulliken": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
        "ldc_potential": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
        "ldc_scf_mix": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_double, c_void_p, P_double]),
        "ldc_cluster_spectrum": (c_int, [c_void_p, c_int, P_double, P_double, P_int]),
        "ldc_last_error": (ctypes.c_char_p, [c_void_p, P_int]),
        "ldc_cluster_dims": (c_int, [c_void_p, P_int]),
        "ldc_profile": (c_int, [c_void_p, c_int]),
        "ldc_stage_times": (c_int, [c_void_p, P_double, P_int]),
        "ldc_stage_name": (ctypes.c_char_p, [c_int]),
        "ldc_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def _ptr(t):
    """Raw device pointer of a torch tensor (or an int address)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _dev(t, n, name, device=None):
    """Device pointer of a float64 tensor of exactly n elements, contiguous, on the plan's GPU.
    Anything else raises before a kernel could read or write out of bounds."""
    if t is None:
        raise LdcError(1, f"{name} is required")
    if isinstance(t, int):
        return t
    import torch
    if not isinstance(t, torch.Tensor):
        raise LdcError(1, f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise LdcError(1, f"{name} must be a device tensor, got {t.device}")
    if device is not None and t.device != device:
        raise LdcError(1, f"{name} is on {t.device}, the plan's stream is on {device}")
    if t.dtype != torch.float64:
        raise LdcError(1, f"{name} must be float64, got {t.dtype}")
    if not t.is_contiguous():
        raise LdcError(1, f"{name} must be contiguous")
    if t.numel() != n:
        raise LdcError(1, f"{name} has {t.numel()} elements, expected {n}")
    return t.data_ptr()


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class Plan:
    """One geometry's clusters and regions plus the device workspaces (ldc_plan_create)."""

    def __init__(self, pos, cell, periodic, n_orb, row_ptr, col, r_L, kappa=0.3, spin_g=2, workgroups=0,
                 stream=None, dist_tol=0.0, shell_tol=0.0, prec="fp64", batched=False, use_graph=False,
                 tune_cache=None):
        lib = load()
        self._lib = lib
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        cell = np.ascontiguousarray(cell, dtype=np.float64)
        periodic = np.ascontiguousarray(periodic, dtype=np.int32)
        n_orb = np.ascontiguousarray(n_orb, dtype=np.int32)
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        col = np.ascontiguousarray(col, dtype=np.int32)
        self.n_atoms = len(n_orb)
        self.n_orb = n_orb
        self._tune_cache = tune_cache.encode() if tune_cache else None  # outlives the plan
        opt = Options(float(r_L), float(kappa), float(dist_tol), float(shell_tol), int(spin_g), int(workgroups),
                      PREC[prec] if isinstance(prec, str) else int(prec), int(bool(batched)), int(bool(use_graph)),
                      self._tune_cache)
        self._device = None
        if stream is not None and not isinstance(stream, int):
            self._device = stream.device
        h = c_void_p()
        st = lib.ldc_plan_create(ctypes.byref(h), self.n_atoms, pos.ctypes.data_as(P_double),
                                 cell.ctypes.data_as(P_double), periodic.ctypes.data_as(P_int),
                                 n_orb.ctypes.data_as(P_int), len(col), row_ptr.ctypes.data_as(P_int),
                                 col.ctypes.data_as(P_int), ctypes.byref(opt), _stream_handle(stream))
        if st != 0:
            raise LdcError(st, "ldc_plan_create failed")
        self._h = h
        inf = self.info()
        self.blk_total = int(inf["blk_total"])

    @classmethod
    def from_system(cls, sysd, **kw):
        """Plan for a system dict with pos, cell, periodic, n_orb, row_ptr, col, r_L (and kappa)."""
        kw.setdefault("kappa", sysd.get("kappa", 0.3))
        kw.setdefault("spin_g", sysd.get("spin_g", 2))
        return cls(sysd["pos"], sysd["cell"], sysd["periodic"], sysd["n_orb"], sysd["row_ptr"], sysd["col"],
                   sysd["r_L"], **kw)

    def _check(self, st):
        if st != 0:
            where = c_int(-1)
            msg = self._lib.ldc_last_error(self._h, ctypes.byref(where))
            raise LdcError(st, msg.decode() if msg else "", where.value)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ldc_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        self._check(self._lib.ldc_plan_set_stream(self._h, _stream_handle(stream)))
        if stream is not None and not isinstance(stream, int):
            self._device = stream.device

    def _m(self, t, name):
        """A block-sparse matrix argument (blk_total float64 values on the plan's GPU)."""
        return _dev(t, self.blk_total, name, self._device)

    def _v(self, t, name):
        """A per-atom vector argument (n_atoms float64 values on the plan's GPU)."""
        return _dev(t, self.n_atoms, name, self._device)

    def buckets(self):
        """Size buckets of the current mode: list of dicts (begin, count, dim_bound, grids)."""
        nb = self.info()["n_buckets"]
        b, c, d = (np.zeros(nb, dtype=np.int32) for _ in range(3))
        g = np.zeros(nb * len(TUNED_STAGES), dtype=np.int32)
        self._check(self._lib.ldc_plan_buckets(self._h, b.ctypes.data_as(P_int), c.ctypes.data_as(P_int),
                                               d.ctypes.data_as(P_int), g.ctypes.data_as(P_int)))
        g = g.reshape(nb, len(TUNED_STAGES))
        return [{"begin": int(b[k]), "count": int(c[k]), "dim_bound": int(d[k]),
                 "grids": dict(zip(TUNED_STAGES, map(int, g[k])))} for k in range(nb)]

    def info(self):
        inf = PlanInfo()
        self._check(self._lib.ldc_plan_query(self._h, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in PlanInfo._fields_}

    def cluster(self, atom):
        """(members, is_long) of an atom's cluster in the library's member order."""
        cap = self.info()["max_members"]
        mem = np.zeros(cap, dtype=np.int32)
        lng = np.zeros(cap, dtype=np.int32)
        nm, nl = c_int(), c_int()
        self._check(self._lib.ldc_plan_cluster(self._h, int(atom), mem.ctypes.data_as(P_int),
                                               lng.ctypes.data_as(P_int), ctypes.byref(nm), ctypes.byref(nl)))
        return mem[: nm.value].copy(), lng[: nm.value].copy()

    def lno(self, S, Dprev, lambda_th=0.1, k_min=1, k_max=-1, fixed_rank=None, want_ranks=True):
        """ldc_lno: LNOs from the previous density (Dprev None -> plain DC).  Returns ranks."""
        ranks = np.zeros(self.n_atoms, dtype=np.int32) if want_ranks else None
        rule, _keep = self._rule(lambda_th, k_min, k_max, fixed_rank, self.n_atoms)
        st = self._lib.ldc_lno(self._h, self._m(S, "S") if Dprev is not None else _ptr(S),
                               self._m(Dprev, "Dprev") if Dprev is not None else None, ctypes.byref(rule),
                               ranks.ctypes.data_as(P_int) if ranks is not None else None)
        self._check(st)
        return ranks

    @staticmethod
    def _rule(lambda_th, k_min, k_max, fixed_rank, n_atoms):
        fr = None
        if fixed_rank is not None:
            fr = np.ascontiguousarray(np.broadcast_to(np.asarray(fixed_rank, dtype=np.int32), (n_atoms,)))
        rule = RankRule(float(lambda_th), int(k_min), int(k_max), fr.ctypes.data_as(P_int) if fr is not None else None)
        return rule, fr

    def build(self, H, S, Dprev, n_electrons, kT, D_out, lambda_th=0.1, k_min=1, k_max=-1, fixed_rank=None):
        """ldc_build: one whole density build (LNOs from Dprev, or plain DC when None), captured
        into a HIP graph and replayed when the plan was made with use_graph.  Returns
        (mu, e_band, n_e)."""
        rule, _keep = self._rule(lambda_th, k_min, k_max, fixed_rank, self.n_atoms)
        mu, eb, ne = c_double(), c_double(), c_double()
        self._check(self._lib.ldc_build(self._h, self._m(H, "H"), self._m(S, "S"),
                                        self._m(Dprev, "Dprev") if Dprev is not None else None, ctypes.byref(rule),
                                        float(n_electrons), float(kT), self._m(D_out, "D_out"), ctypes.byref(mu),
                                        ctypes.byref(eb), ctypes.byref(ne)))
        return mu.value, eb.value, ne.value

    def tune(self, H, S, Dprev, n_electrons, kT, D_out, lambda_th=0.1, k_min=1, k_max=-1, fixed_rank=None):
        """ldc_tune: pick size buckets and per-bucket launch grids by timing whole builds; writes
        the plan's tuning cache when it has one.  Returns the tuned build time (ms)."""
        rule, _keep = self._rule(lambda_th, k_min, k_max, fixed_rank, self.n_atoms)
        ms = c_double()
        self._check(self._lib.ldc_tune(self._h, self._m(H, "H"), self._m(S, "S"),
                                       self._m(Dprev, "Dprev") if Dprev is not None else None, ctypes.byref(rule),
                                       float(n_electrons), float(kT), self._m(D_out, "D_out"), ctypes.byref(ms)))
        return ms.value

    def reference_populations(self, n_electrons, q0_out):
        """ldc_reference_populations: q0_i = N_e M_i / sum_j M_j into the device vector q0_out."""
        self._check(self._lib.ldc_reference_populations(self._h, float(n_electrons), self._v(q0_out, "q0_out")))

    def solve(self, H, S):
        """ldc_solve: gather + batched generalized eigensolve of every cluster."""
        self._check(self._lib.ldc_solve(self._h, self._m(H, "H"), self._m(S, "S")))

    def density(self, n_electrons, kT, D_out):
        """ldc_density: mu by bisection and density rows into D_out.  Returns (mu, e_band, n_e)."""
        mu, eb, ne = c_double(), c_double(), c_double()
        self._check(self._lib.ldc_density(self._h, float(n_electrons), float(kT), self._m(D_out, "D_out"),
                                          ctypes.byref(mu),
                                          ctypes.byref(eb), ctypes.byref(ne)))
        return mu.value, eb.value, ne.value

    def density_noalloc(self, n_electrons, kT, D_out, result_out):
        """ldc_density_noalloc: as density(), with no allocation and no wait for the device; mu,
        e_band and n_e go to the device vector result_out (3 float64)."""
        self._check(self._lib.ldc_density_noalloc(self._h, float(n_electrons), float(kT), self._m(D_out, "D_out"),
                                                  _dev(result_out, 3, "result_out", self._device)))

    def density_at(self, mu, kT, D_out):
        """ldc_density_at: density rows at a given chemical potential.  Returns (e_band, n_e)."""
        eb, ne = c_double(), c_double()
        self._check(self._lib.ldc_density_at(self._h, float(mu), float(kT), self._m(D_out, "D_out"),
                                             ctypes.byref(eb),
                                             ctypes.byref(ne)))
        return eb.value, ne.value

    def energy_density(self, E_out):
        """ldc_energy_density: energy density rows (Eq. 25) at the last density's mu into E_out.
        Returns g Tr(E S)."""
        tr = c_double()
        self._check(self._lib.ldc_energy_density(self._h, self._m(E_out, "E_out"), ctypes.byref(tr)))
        return tr.value

    def window_density(self, e_lo, e_hi, kT, W_out):
        """ldc_window_density: energy-window density rows over (e_lo, e_hi) with edge width kT into
        W_out.  Returns g Tr(W S)."""
        tr = c_double()
        self._check(self._lib.ldc_window_density(self._h, float(e_lo), float(e_hi), float(kT), self._m(W_out, "W_out"),
                                                 ctypes.byref(tr)))
        return tr.value

    def mulliken(self, D, S, q_out):
        """ldc_mulliken: Mulliken populations of every atom from the density rows into q_out."""
        self._check(self._lib.ldc_mulliken(self._h, self._m(D, "D"), self._m(S, "S"), self._v(q_out, "q_out")))

    def potential(self, H0, S, v, H_out):
        """ldc_potential: H_out = H0 + (v_i + v_j)/2 S on every pattern block."""
        self._check(self._lib.ldc_potential(self._h, self._m(H0, "H0"), self._m(S, "S"), self._v(v, "v"),
                                            self._m(H_out, "H_out")))

    def scf_mix(self, q_out, q_in, q0, U, alpha, v_out, want_residual=True):
        """ldc_scf_mix: q_in += alpha (q_out - q_in), v_out = U (q_in - q0).  Returns the residual
        max |q_out - q_in| (before the mixing) when want_residual, else None."""
        res = c_double()
        self._check(self._lib.ldc_scf_mix(self._h, self._v(q_out, "q_out"), self._v(q_in, "q_in"), self._v(q0, "q0"),
                                          float(U), float(alpha), self._v(v_out, "v_out"),
                                          ctypes.byref(res) if want_residual else None))
        return res.value if want_residual else None

    def cluster_dims(self):
        """Reduced dimension of every cluster after the last solve."""
        d = np.zeros(self.n_atoms, dtype=np.int32)
        self._check(self._lib.ldc_cluster_dims(self._h, d.ctypes.data_as(P_int)))
        return d

    def profile(self, enable=True):
        """Enable (and reset) or disable per-stage HIP-event timing."""
        self._check(self._lib.ldc_profile(self._h, 1 if enable else 0))

    def stage_times(self):
        """({stage name: ms summed over builds}, builds) since profiling was enabled."""
        ms = np.zeros(NUM_STAGES)
        b = c_int()
        self._check(self._lib.ldc_stage_times(self._h, ms.ctypes.data_as(P_double), ctypes.byref(b)))
        return {self._lib.ldc_stage_name(i).decode(): float(ms[i]) for i in range(NUM_STAGES)}, b.value

    def cluster_spectrum(self, atom):
        """(eps, w) of one cluster, copied to the host."""
        cap = self.info()["max_dim_pao"]
        eps = np.zeros(cap)
        w = np.zeros(cap)
        dim = c_int()
        self._check(self._lib.ldc_cluster_spectrum(self._h, int(atom), eps.ctypes.data_as(P_double),
                                                   w.ctypes.data_as(P_double), ctypes.byref(dim)))
        return eps[: dim.value].copy(), w[: dim.value].copy()


def regions(pos, cell, periodic, n_orb, row_ptr, col, r_L, kappa=0.3, dist_tol=0.0, shell_tol=0.0):
    """Host-only planner (ldc_regions): (member_ptr, members, is_long) in the library's order."""
    lib = load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    cell = np.ascontiguousarray(cell, dtype=np.float64)
    periodic = np.ascontiguousarray(periodic, dtype=np.int32)
    n_orb = np.ascontiguousarray(n_orb, dtype=np.int32)
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    n = len(n_orb)
    opt = Options(float(r_L), float(kappa), float(dist_tol), float(shell_tol), 2, 0)
    ptr = np.zeros(n + 1, dtype=np.int32)
    cap = 0
    for attempt in range(2):
        mem = np.zeros(max(cap, 1), dtype=np.int32)
        lng = np.zeros(max(cap, 1), dtype=np.int32)
        st = lib.ldc_regions(n, pos.ctypes.data_as(P_double), cell.ctypes.data_as(P_double),
                             periodic.ctypes.data_as(P_int), n_orb.ctypes.data_as(P_int), len(col),
                             row_ptr.ctypes.data_as(P_int), col.ctypes.data_as(P_int), ctypes.byref(opt), cap,
                             ptr.ctypes.data_as(P_int), mem.ctypes.data_as(P_int), lng.ctypes.data_as(P_int))
        if st == 0:
            return ptr, mem[: ptr[-1]], lng[: ptr[-1]]
        if st != 9:
            raise LdcError(st, "ldc_regions failed")
        cap = int(ptr[-1])
    raise LdcError(9, "ldc_regions capacity")


def version():
    return load().ldc_version().decode()
