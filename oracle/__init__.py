"""Python access to the FP64 CPU oracle (oracle/ngravs_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg. The GPU library never imports this package and
this package never imports the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborcngravs.so")
SOURCES = [os.path.join(HERE, "ngravs_oracle.c")]

GRID = {"r": 0, "r2": 1}
PRUNE, ACCEPT, OPEN = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11, OpenMP, no fused multiply-add)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-Wall", "-Wno-unknown-pragmas", *SOURCES, "-lm", "-o", LIB_PATH + ".tmp"]
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        u64, u32, i32, dbl = C.c_uint64, C.c_uint32, C.c_int32, C.c_double
        sig = {
            "orc_num_threads": (C.c_int, []),
            "orc_lattice": (None, [u64, P, dbl, P]),
            "orc_morton": (u64, [u32, u32, u32]),
            "orc_hilbert": (u64, [u32, u32, u32]),
            "orc_hilbert_decode": (None, [u64, P]),
            "orc_keys_order": (None, [u64, P, P, u32, P]),
            "orc_tree_build_order": (P, [u64, u32, dbl, P, P, P, u32, u32]),
            "orc_keys": (None, [u64, P, P, P]),
            "orc_sort": (None, [u64, P, P]),
            "orc_tree_build": (P, [u64, u32, dbl, P, P, P, u32]),
            "orc_tree_free": (None, [P]),
            "orc_tree_n_nodes": (u64, [P]),
            "orc_tree_export": (None, [P] * 10),
            "orc_monopoles": (None, [P]),
            "orc_monopoles_export": (None, [P, P, P]),
            "orc_groups": (u64, [P, u32]),
            "orc_groups_export": (None, [P] * 6),
            "orc_mac": (C.c_int, [P, u64, P, P, dbl, dbl]),
            "orc_mac_relative": (C.c_int, [P, u64, P, P, dbl, dbl, dbl]),
            "orc_group_list": (u64, [P, P, u64, P, u64]),
            "orc_tree_force": (C.c_int, [P, P, P, u64, P, P, P, P]),
            "orc_direct": (C.c_int, [u64, u32, dbl, P, P, P, P, P, u64, P, P]),
            "orc_factor": (dbl, [P, u32, u32, dbl, dbl]),
            "orc_cored_radial": (dbl, [dbl, dbl]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _ = i32
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


LAW_TABLE, LAW_ACCUMULATOR = 0, 1
OPEN_GEOMETRIC, OPEN_RELATIVE = 0, 1


class Law(C.Structure):
    _fields_ = [("G", C.c_void_p), ("tables", C.c_void_p), ("ntab", C.c_uint32),
                ("grid", C.c_uint32), ("r_cut", C.c_double), ("eps", C.c_double),
                ("theta", C.c_double), ("kind", C.c_uint32), ("cored", C.c_uint32),
                ("beta", C.c_double), ("track_counts", C.c_uint32), ("eps_ab", C.c_void_p),
                ("opening", C.c_uint32), ("alpha", C.c_double), ("old_acc", C.c_void_p),
                ("corr", C.c_void_p), ("corr_n", C.c_uint32)]


def make_law(G, tables, grid, r_cut, eps, theta, kind=LAW_TABLE, cored=(), beta=0.0, track_counts=True,
             eps_ab=None, alpha=None, old_acc=None, corr=None):
    """cored: species indices with a core (accumulator laws); eps_ab: D x D
    per-pair softening, or None for eps everywhere; alpha and old_acc (n
    previous |a| in input order) select the relative opening test; corr
    (D, D, n+1, n+1, n+1, 3) lattice correction tables (no cut-off then)."""
    G = np.ascontiguousarray(G, dtype=np.float64)
    tables = np.ascontiguousarray(tables, dtype=np.float64)
    ea = None if eps_ab is None else np.ascontiguousarray(eps_ab, dtype=np.float64)
    mask = 0
    for b in cored:
        mask |= 1 << int(b)
    law = Law(G.ctypes.data, tables.ctypes.data, tables.shape[-1], GRID[grid],
              float(r_cut), float(eps), float(theta), int(kind), mask, float(beta), int(bool(track_counts)),
              None if ea is None else ea.ctypes.data)
    oa = None
    if alpha is not None:
        oa = np.ascontiguousarray(old_acc, dtype=np.float64)
        law.opening, law.alpha, law.old_acc = OPEN_RELATIVE, float(alpha), oa.ctypes.data
    co = None
    if corr is not None:
        co = np.ascontiguousarray(corr, dtype=np.float64)
        law.corr, law.corr_n = co.ctypes.data, co.shape[2] - 1
    law._keep = (G, tables, ea, oa, co)  # keep the buffers alive with the struct
    return law


def law_of(p, track_counts=True):
    acc = getattr(p, "accumulator", None)
    eps_ab = getattr(p, "eps_ab", None)
    rel = getattr(p, "relative", None)
    extra = dict(eps_ab=eps_ab, corr=getattr(p, "lattice_corr", None))
    if rel is not None:
        extra.update(alpha=rel["alpha"], old_acc=rel["old_acc"])
    if acc is None:
        return make_law(p.G, p.tables, p.grid, p.r_cut, p.eps, p.theta, **extra)
    return make_law(p.G, p.tables, p.grid, p.r_cut, p.eps, p.theta, kind=LAW_ACCUMULATOR,
                    cored=acc["cored"], beta=acc["beta"], track_counts=track_counts, **extra)


def cored_radial(r: float, s: float) -> float:
    """orc_cored_radial: the accumulator laws' radial factor (see the C source)."""
    return float(lib().orc_cored_radial(float(r), float(s)))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def lattice(x: np.ndarray, box: float) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    X = np.empty(x.shape, dtype=np.uint64)
    lib().orc_lattice(x.shape[-1], _p(x), box, _p(X))
    return X


def box_of(p) -> float:
    """The lattice's box: the problem's own, or for a non-periodic problem
    four times it, where every minimum-image difference of two particles in
    [0, box) is their plain difference (the non-periodic reading)."""
    return p.box if getattr(p, "periodic", True) else 4.0 * p.box


def lattice_of(p) -> np.ndarray:
    if p.lattice is not None:
        return np.ascontiguousarray(p.lattice, dtype=np.uint64)
    return lattice(p.pos, box_of(p))


def morton(kx: int, ky: int, kz: int) -> int:
    return int(lib().orc_morton(kx, ky, kz))


KEY_ORDER = {"morton": 0, "hilbert": 1}


def hilbert(kx: int, ky: int, kz: int) -> int:
    return int(lib().orc_hilbert(kx, ky, kz))


def hilbert_decode(h: int):
    k = np.zeros(3, np.uint32)
    lib().orc_hilbert_decode(int(h), _p(k))
    return tuple(int(v) for v in k)


def keys(X: np.ndarray, species: np.ndarray, key_order: str = "morton") -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.uint64)
    s = np.ascontiguousarray(species, dtype=np.uint8)
    K = np.empty(s.shape[0], dtype=np.uint64)
    lib().orc_keys_order(s.shape[0], _p(X), _p(s), KEY_ORDER[key_order], _p(K))
    return K


def sort(K: np.ndarray) -> np.ndarray:
    K = np.ascontiguousarray(K, dtype=np.uint64)
    perm = np.empty(K.shape[0], dtype=np.uint32)
    lib().orc_sort(K.shape[0], _p(K), _p(perm))
    return perm


def factor(T: np.ndarray, grid: str, r2: float, r_cut: float) -> float:
    T = np.ascontiguousarray(T, dtype=np.float64)
    return float(lib().orc_factor(_p(T), T.shape[0], GRID[grid], r2, r_cut))


class Tree:
    """The oracle's tree over one particle set (lattice positions)."""

    def __init__(self, X, species, mass, D: int, box: float, leaf_size: int = 16, key_order: str = "morton"):
        self.X = np.ascontiguousarray(X, dtype=np.uint64)
        self.species = np.ascontiguousarray(species, dtype=np.uint8)
        self.mass = np.ascontiguousarray(mass, dtype=np.float64)
        self.n = int(self.species.shape[0])
        self.D, self.box = int(D), float(box)
        self._t = lib().orc_tree_build_order(self.n, self.D, self.box, _p(self.X), _p(self.species),
                                             _p(self.mass), int(leaf_size), KEY_ORDER[key_order])
        self.n_nodes = int(lib().orc_tree_n_nodes(self._t))
        self._mono = False
        self.n_groups = None

    @classmethod
    def of(cls, p, group_size: Optional[int] = None):
        t = cls(lattice_of(p), p.species, p.mass, p.D, box_of(p), p.leaf_size, getattr(p, "key_order", "morton"))
        t.monopoles()
        t.groups(p.group_size if group_size is None else group_size)
        return t

    def __del__(self):
        t = getattr(self, "_t", None)
        if t and _lib is not None:
            try:
                _lib.orc_tree_free(t)
            except Exception:
                pass
            self._t = None

    def nodes(self) -> dict:
        nn, D, n = self.n_nodes, self.D, self.n
        out = dict(perm=np.empty(n, np.uint32), keys=np.empty(n, np.uint64),
                   level=np.empty(nn, np.uint8), prefix=np.empty(nn, np.uint64),
                   parent=np.empty(nn, np.int32), first_child=np.empty(nn, np.int32),
                   n_child=np.empty(nn, np.uint8), start=np.empty((D, nn), np.uint32),
                   count=np.empty((D, nn), np.uint32))
        lib().orc_tree_export(self._t, *[_p(out[k]) for k in
                                         ("perm", "keys", "level", "prefix", "parent",
                                          "first_child", "n_child", "start", "count")])
        return out

    def monopoles(self):
        lib().orc_monopoles(self._t)
        self._mono = True

    def monopole_arrays(self):
        M = np.empty((self.D, self.n_nodes))
        com = np.empty((self.D, 3, self.n_nodes))
        lib().orc_monopoles_export(self._t, _p(M), _p(com))
        return M, com

    def groups(self, group_size: int) -> int:
        self.n_groups = int(lib().orc_groups(self._t, int(group_size)))
        return self.n_groups

    def group_arrays(self) -> dict:
        ng = self.n_groups
        out = dict(species=np.empty(ng, np.uint8), start=np.empty(ng, np.uint32),
                   count=np.empty(ng, np.uint32), lo=np.empty((3, ng), np.uint32),
                   hi=np.empty((3, ng), np.uint32))
        lib().orc_groups_export(self._t, *[_p(out[k]) for k in ("species", "start", "count", "lo", "hi")])
        return out

    def mac(self, node: int, lo, hi, R2: float, theta2: float) -> int:
        lo = np.ascontiguousarray(lo, np.uint32)
        hi = np.ascontiguousarray(hi, np.uint32)
        return int(lib().orc_mac(self._t, node, _p(lo), _p(hi), R2, theta2))

    def mac_relative(self, node: int, lo, hi, R2: float, rel_k: float, a_min: float) -> int:
        lo = np.ascontiguousarray(lo, np.uint32)
        hi = np.ascontiguousarray(hi, np.uint32)
        return int(lib().orc_mac_relative(self._t, node, _p(lo), _p(hi), R2, rel_k, a_min))

    def group_list(self, law, g: int) -> np.ndarray:
        n = int(lib().orc_group_list(self._t, C.byref(law), g, None, 0))
        e = np.empty(max(n, 1), np.uint64)
        lib().orc_group_list(self._t, C.byref(law), g, _p(e), n)
        return e[:n]

    def force(self, law, groups: Optional[np.ndarray] = None, group_counts: bool = False):
        """Tree force. Returns (acc (3, n) in input order, slack (n,), counts
        {'pp', 'pn', 'near_ties', 'pn_species'}, per-group counts or None).
        Rows of sinks outside the listed groups are NaN."""
        n = self.n
        acc = np.full((3, n), np.nan)
        slack = np.full(n, np.nan)
        cnt = np.zeros(3 + 6, np.uint64)
        gsel = None if groups is None else np.ascontiguousarray(groups, np.uint32)
        nsel = self.n_groups if gsel is None else gsel.shape[0]
        gc = np.zeros((nsel, 4), np.uint64) if group_counts else None
        rc = lib().orc_tree_force(self._t, C.byref(law), _p(gsel), 0 if gsel is None else nsel,
                                  _p(acc), _p(slack), _p(cnt), _p(gc))
        if rc != 0:
            raise RuntimeError("oracle tree force failed")
        return acc, slack, {"pp": int(cnt[0]), "pn": int(cnt[1]), "near_ties": int(cnt[2]),
                            "pn_species": [int(c) for c in cnt[3:3 + self.D]]}, gc


def direct(X, species, mass, D: int, box: float, law, sinks: Optional[np.ndarray] = None):
    """Minimum-image direct sum for the given sinks (input indices, default
    all). Returns (acc (3, n_sinks), slack (n_sinks,))."""
    X = np.ascontiguousarray(X, dtype=np.uint64)
    s = np.ascontiguousarray(species, dtype=np.uint8)
    m = np.ascontiguousarray(mass, dtype=np.float64)
    n = s.shape[0]
    sinks = np.arange(n, dtype=np.uint32) if sinks is None else np.ascontiguousarray(sinks, np.uint32)
    acc = np.empty((3, sinks.shape[0]))
    slack = np.empty(sinks.shape[0])
    lib().orc_direct(n, D, box, _p(X), _p(s), _p(m), C.byref(law), _p(sinks), sinks.shape[0],
                     _p(acc), _p(slack))
    return acc, slack


def direct_of(p, sinks=None):
    return direct(lattice_of(p), p.species, p.mass, p.D, box_of(p), law_of(p), sinks)
