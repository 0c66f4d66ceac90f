"""Python binding of libngravs (include/ngravs.h): argument marshalling only.

Every step of the force computation runs in the HIP kernels of the shared
library; this module only turns torch device tensors and numpy host arrays
into the pointers and sizes of the C-ABI, on torch's current HIP stream.
There is no CPU fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libngravs.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE = 0, -1, -2, -3, -4
GRID_R, GRID_R2 = 0, 1
GRIDS = {"r": GRID_R, "r2": GRID_R2, GRID_R: GRID_R, GRID_R2: GRID_R2}
MAX_SPECIES = 6
EXPORTED = ["ngr_context_create", "ngr_context_destroy", "ngr_last_error", "ngr_tree_build",
            "ngr_compute_monopoles", "ngr_tree_force", "ngr_tree_force_counts", "ngr_tree_force_noalloc",
            "ngr_tree_free",
            "ngr_tree_info", "ngr_tree_export", "ngr_monopoles_export", "ngr_groups_export",
            "ngr_batch_build_force", "ngr_server_create", "ngr_server_submit", "ngr_server_tick",
            "ngr_server_status", "ngr_server_take", "ngr_server_destroy", "ngr_short_range_grid",
            "ngr_short_range_tables", "ngr_pm_create", "ngr_pm_force", "ngr_pm_destroy", "ngr_autotune",
            "ngr_tuned_group_size"]


class NgravsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"ngravs status {status}: {msg}")
        self.status = status


class Particles(C.Structure):
    _fields_ = [("n", C.c_uint64), ("D", C.c_uint32), ("box", C.c_double), ("pos", C.c_void_p),
                ("lattice", C.c_void_p), ("species", C.c_void_p), ("mass", C.c_void_p)]


KEY_ORDER = {"morton": 0, "hilbert": 1}     # NGR_KEY_MORTON, NGR_KEY_HILBERT


class TreeParams(C.Structure):
    _fields_ = [("leaf_size", C.c_uint32), ("non_periodic", C.c_uint32), ("key_order", C.c_uint32)]


class ForceParams(C.Structure):
    _fields_ = [("G", C.c_void_p), ("tables", C.c_void_p), ("ntab", C.c_uint32), ("grid", C.c_uint32),
                ("r_s", C.c_double), ("r_cut", C.c_double), ("eps", C.c_double), ("theta", C.c_double),
                ("group_size", C.c_uint32), ("law", C.c_uint32), ("cored", C.c_uint32), ("beta", C.c_double),
                ("eps_ab", C.c_void_p), ("opening", C.c_uint32), ("alpha", C.c_double), ("old_acc", C.c_void_p),
                ("lattice_corr", C.c_void_p), ("corr_n", C.c_uint32), ("tables_on_device", C.c_uint32)]


NOT_COUNTED = 2 ** 64 - 1     # NGR_NOT_COUNTED


class ForceStats(C.Structure):
    _fields_ = [("interactions_pp", C.c_uint64), ("interactions_pn", C.c_uint64), ("n_nodes", C.c_uint64),
                ("n_leaves", C.c_uint64), ("n_groups", C.c_uint64), ("group_size", C.c_uint32),
                ("depth", C.c_uint32), ("ms_groups", C.c_double), ("ms_walk", C.c_double),
                ("interactions_pn_species", C.c_uint64 * 6), ("near_ties", C.c_uint64),
                ("ms_build", C.c_double), ("ms_build_ingest", C.c_double), ("ms_build_sort", C.c_double),
                ("ms_build_octree", C.c_double), ("ms_monopoles", C.c_double)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["interactions_pn_species"] = list(d["interactions_pn_species"])
        return d


class Box(C.Structure):
    _fields_ = [("particles", Particles), ("tree", TreeParams), ("force", ForceParams), ("acc", C.c_void_p)]


class RequestDesc(C.Structure):
    _fields_ = [("particles", Particles), ("vel", C.c_void_p), ("tree", TreeParams), ("force", ForceParams),
                ("dt", C.c_double), ("steps", C.c_uint32)]


class TuneStats(C.Structure):
    _fields_ = [("classes", C.c_uint32), ("launches", C.c_uint32), ("ms", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


def autotune(ctx: Context, boxes) -> dict:
    """ngr_autotune over a list of BatchBox: afterwards group_size = 0
    resolves to the fastest measured size of each box's class."""
    arr = (Box * len(boxes))()
    for k, b in enumerate(boxes):
        arr[k] = Box(b.particles, b.tree, b.force, b.acc)
    st = TuneStats()
    ctx._check(lib().ngr_autotune(ctx.handle, len(boxes), arr, C.byref(st)), "autotune")
    return st.as_dict()


def tuned_group_size(ctx: Context, n: int, D: int) -> int:
    gs = C.c_uint32()
    rc = lib().ngr_tuned_group_size(ctx.handle, int(n), int(D), C.byref(gs))
    if rc != 0:
        raise NgravsError(rc, "tuned_group_size: bad arguments")
    return gs.value


class ServerParams(C.Structure):
    _fields_ = [("hbm_budget", C.c_uint64), ("max_active", C.c_uint32)]


class TickStats(C.Structure):
    _fields_ = [("admitted", C.c_uint32), ("evaluated", C.c_uint32), ("finished", C.c_uint32), ("active", C.c_uint32),
                ("pending", C.c_uint32), ("particles", C.c_uint64), ("interactions", C.c_uint64),
                ("resident_bytes", C.c_uint64), ("ms", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class BatchStats(C.Structure):
    _fields_ = [("n_particles", C.c_uint64), ("n_nodes", C.c_uint64), ("n_groups", C.c_uint64),
                ("interactions_pp", C.c_uint64), ("interactions_pn", C.c_uint64), ("ms_build", C.c_double),
                ("ms_monopoles", C.c_double), ("ms_groups", C.c_double), ("ms_walk", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load libngravs.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        P, u64, u32, i32 = C.c_void_p, C.c_uint64, C.c_uint32, C.c_int32
        sig = {
            "ngr_context_create": (i32, [C.c_int, P, P]),
            "ngr_context_destroy": (None, [P]),
            "ngr_last_error": (C.c_char_p, [P]),
            "ngr_tree_build": (i32, [P, P, P, P]),
            "ngr_compute_monopoles": (i32, [P, P, C.c_int]),
            "ngr_tree_force": (i32, [P, P, P, P, P]),
            "ngr_tree_force_counts": (i32, [P, P, P, P, P, P]),
            "ngr_tree_force_noalloc": (i32, [P, P, P, P, P]),
            "ngr_tree_free": (i32, [P, P]),
            "ngr_tree_info": (i32, [P, P, P, P, P]),
            "ngr_tree_export": (i32, [P] * 12),
            "ngr_monopoles_export": (i32, [P] * 4),
            "ngr_groups_export": (i32, [P, P, u32, P, P, P, P, P, P]),
            "ngr_batch_build_force": (i32, [P, u32, P, P, P]),
            "ngr_server_create": (i32, [P, P, P]),
            "ngr_server_submit": (i32, [P, P, P]),
            "ngr_server_tick": (i32, [P, P]),
            "ngr_server_status": (i32, [P, u64, P, P]),
            "ngr_server_take": (i32, [P, u64, P, P, P]),
            "ngr_server_destroy": (None, [P]),
            "ngr_short_range_grid": (i32, [C.c_double, C.c_double, C.c_double, P, P]),
            "ngr_short_range_tables": (i32, [P, P, P, P, P]),
            "ngr_pm_create": (i32, [P, P, P, P, P]),
            "ngr_pm_force": (i32, [P, P, P, P, C.c_int, P]),
            "ngr_pm_destroy": (i32, [P, P]),
            "ngr_autotune": (i32, [P, u32, P, P]),
            "ngr_tuned_group_size": (i32, [P, u64, u32, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype, f.argtypes = res, args
        _ = u64
        _lib = L
    return _lib


def _np(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _dev(t) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return t.data_ptr()


class Context:
    """A library context on one HIP device, bound to a HIP stream (default:
    torch's current stream on that device)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        handle = stream if isinstance(stream, int) else stream.cuda_stream
        self._h = C.c_void_p()
        self._check(lib().ngr_context_create(device, C.c_void_p(handle), C.byref(self._h)), "context create")
        self.device = device

    def _check(self, status: int, what: str):
        if status != OK:
            msg = lib().ngr_last_error(self._h).decode() if getattr(self, "_h", None) else what
            raise NgravsError(status, msg or what)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().ngr_context_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tree:
    def __init__(self, ctx: Context, handle: C.c_void_p):
        self.ctx, self._h = ctx, handle
        n, nn, D, depth = C.c_uint64(), C.c_uint64(), C.c_uint32(), C.c_uint32()
        lib().ngr_tree_info(handle, C.byref(n), C.byref(nn), C.byref(D), C.byref(depth))
        self.n, self.n_nodes, self.D, self.depth = n.value, nn.value, D.value, depth.value

    @property
    def handle(self):
        return self._h


def tree_build(ctx: Context, *, D: int, box: float, species, mass, pos=None, lattice=None,
               leaf_size: int = 16, periodic: bool = True, key_order: str = "morton") -> Tree:
    """ngr_tree_build: device tensors species (uint8, n), mass (float64, n) and
    either pos (float64, 3 x n) or lattice (uint64 lattice as int64, 3 x n).
    periodic=False: a non-periodic box (positions in [0, box)^3 only);
    key_order "morton" or "hilbert" (the Peano-Hilbert curve)."""
    n = int(species.shape[0])
    p = Particles(n, D, float(box), _dev(pos), _dev(lattice), _dev(species), _dev(mass))
    tp = TreeParams(leaf_size, 0 if periodic else 1, KEY_ORDER[key_order])
    h = C.c_void_p()
    ctx._check(lib().ngr_tree_build(ctx.handle, C.byref(p), C.byref(tp), C.byref(h)), "tree build")
    return Tree(ctx, h)


def compute_monopoles(ctx: Context, tree: Tree, track_counts: bool = True):
    ctx._check(lib().ngr_compute_monopoles(ctx.handle, tree.handle, int(track_counts)), "monopoles")


LAW_TABLE, LAW_ACCUMULATOR = 0, 1


def _force_params(D, G, tables, grid, r_s, r_cut, eps, theta, group_size, ntab=None, accumulator=None,
                  eps_ab=None, relative=None, lattice_corr=None):
    """accumulator: None for a table law, else {"cored": species indices,
    "beta": beta} for the accumulator laws; eps_ab: D x D per-pair softening
    or None; relative: None for the geometric opening test, else {"alpha":
    alpha, "old_acc": device tensor of the previous |a| (n, float64)};
    lattice_corr: host (D, D, n+1, n+1, n+1, 3) correction tables or None.
    tables: a host array, or a contiguous float64 device tensor of
    D x D x ntab samples (read in place by the library)."""
    G = np.ascontiguousarray(G, dtype=np.float64).reshape(D, D)
    on_device = tables is not None and bool(getattr(tables, "is_cuda", False))
    if on_device:
        if str(tables.dtype) != "torch.float64" or not tables.is_contiguous() or tables.numel() % (D * D):
            raise ValueError("device tables must be a contiguous float64 tensor of D x D x ntab samples")
        ntab = tables.numel() // (D * D)
        tables_ptr = tables.data_ptr()
    elif tables is not None:
        tables = np.ascontiguousarray(tables, dtype=np.float64).reshape(D, D, -1)
        ntab = tables.shape[-1]
        tables_ptr = tables.ctypes.data
    law, mask, beta = LAW_TABLE, 0, 0.0
    if accumulator is not None:
        law, beta = LAW_ACCUMULATOR, float(accumulator["beta"])
        for b in accumulator["cored"]:
            mask |= 1 << int(b)
    fp = ForceParams(G.ctypes.data, None if tables is None else tables_ptr, int(ntab), GRIDS.get(grid, grid),
                     float(r_s), float(r_cut), float(eps), float(theta), int(group_size), law, mask, beta)
    fp.tables_on_device = 1 if on_device else 0
    ea = None
    if eps_ab is not None:
        ea = np.ascontiguousarray(eps_ab, dtype=np.float64).reshape(D, D)
        fp.eps_ab = ea.ctypes.data
    oa = None
    if relative is not None:
        oa = relative["old_acc"]
        fp.opening, fp.alpha, fp.old_acc = 1, float(relative["alpha"]), _dev(oa)
    lc = None
    if lattice_corr is not None:
        lc = np.ascontiguousarray(lattice_corr, dtype=np.float64)
        fp.lattice_corr, fp.corr_n = lc.ctypes.data, lc.shape[2] - 1
    fp._keep = (G, tables, ea, oa, lc)
    return fp


def tree_force(ctx: Context, tree: Tree, *, G, tables, grid, r_cut, eps, theta, acc, r_s: float = 0.0,
               group_size: int = 64, ntab: Optional[int] = None, group_counts: bool = False, accumulator=None,
               eps_ab=None, relative=None, lattice_corr=None):
    """ngr_tree_force into the device tensor acc (float64, 3 x n, input order).
    G (D x D) is a host array; tables (D x D x ntab) a host array, a float64
    device tensor (read in place), or None;
    accumulator {"cored": [...], "beta": b} selects the accumulator laws.
    Returns the statistics as a dict (and per-group counts when asked)."""
    fp = _force_params(tree.D, G, tables, grid, r_s, r_cut, eps, theta, group_size, ntab, accumulator, eps_ab,
                       relative, lattice_corr)
    st = ForceStats()
    if group_counts:
        ng = groups_count(ctx, tree, group_size)
        gc = np.zeros((max(ng, 1), 4), np.uint64)
        ctx._check(lib().ngr_tree_force_counts(ctx.handle, tree.handle, C.byref(fp), C.c_void_p(_dev(acc)),
                                               C.byref(st), _np(gc)), "tree force")
        return st.as_dict(), gc[:ng]
    ctx._check(lib().ngr_tree_force(ctx.handle, tree.handle, C.byref(fp), C.c_void_p(_dev(acc)), C.byref(st)),
               "tree force")
    return st.as_dict()


NOALLOC_MAX_N = 1 << 20     # NGR_NOALLOC_MAX_N


def tree_force_noalloc(ctx: Context, tree: Tree, *, G, tables, grid, r_cut, eps, theta, acc, r_s: float = 0.0,
                       group_size: int = 64, ntab: Optional[int] = None, accumulator=None, eps_ab=None,
                       relative=None, lattice_corr=None):
    """ngr_tree_force_noalloc: as tree_force, with the call's scratch in the
    library's static device array (no device allocation). Returns the
    statistics as a dict."""
    fp = _force_params(tree.D, G, tables, grid, r_s, r_cut, eps, theta, group_size, ntab, accumulator, eps_ab,
                       relative, lattice_corr)
    st = ForceStats()
    ctx._check(lib().ngr_tree_force_noalloc(ctx.handle, tree.handle, C.byref(fp), C.c_void_p(_dev(acc)),
                                            C.byref(st)), "tree force (no allocation)")
    return st.as_dict()


def tree_free(ctx: Context, tree: Tree):
    if tree._h:
        ctx._check(lib().ngr_tree_free(ctx.handle, tree.handle), "tree free")
        tree._h = None


def tree_export(ctx: Context, tree: Tree) -> dict:
    n, nn, D = tree.n, tree.n_nodes, tree.D
    out = dict(perm=np.empty(n, np.uint32), keys=np.empty(n, np.uint64), lattice=np.empty((3, n), np.uint64),
               level=np.empty(nn, np.uint8), prefix=np.empty(nn, np.uint64), parent=np.empty(nn, np.int32),
               first_child=np.empty(nn, np.int32), n_child=np.empty(nn, np.uint8),
               start=np.empty((D, nn), np.uint32), count=np.empty((D, nn), np.uint32))
    ctx._check(lib().ngr_tree_export(ctx.handle, tree.handle, *[_np(out[k]) for k in
                                     ("perm", "keys", "lattice", "level", "prefix", "parent", "first_child",
                                      "n_child", "start", "count")]), "tree export")
    return out


def monopoles_export(ctx: Context, tree: Tree):
    M = np.empty((tree.D, tree.n_nodes))
    com = np.empty((tree.D, 3, tree.n_nodes))
    ctx._check(lib().ngr_monopoles_export(ctx.handle, tree.handle, _np(M), _np(com)), "monopoles export")
    return M, com


def groups_count(ctx: Context, tree: Tree, group_size: int = 64) -> int:
    ng = C.c_uint64()
    ctx._check(lib().ngr_groups_export(ctx.handle, tree.handle, group_size, C.byref(ng), None, None, None, None,
                                       None), "groups export")
    return ng.value


def groups_export(ctx: Context, tree: Tree, group_size: int = 64) -> dict:
    ng = groups_count(ctx, tree, group_size)
    out = dict(species=np.empty(ng, np.uint8), start=np.empty(ng, np.uint32), count=np.empty(ng, np.uint32),
               lo=np.empty((3, ng), np.uint32), hi=np.empty((3, ng), np.uint32))
    n2 = C.c_uint64()
    ctx._check(lib().ngr_groups_export(ctx.handle, tree.handle, group_size, C.byref(n2),
                                       *[_np(out[k]) for k in ("species", "start", "count", "lo", "hi")]),
               "groups export")
    return out


class ShortParams(C.Structure):
    _fields_ = [("D", C.c_uint32), ("ntab", C.c_uint32), ("grid", C.c_uint32), ("nk", C.c_uint32),
                ("r_s", C.c_double), ("r_cut", C.c_double), ("dk", C.c_double)]


def short_range_grid(r_s: float, r_cut: float, range_: float = 0.0):
    """ngr_short_range_grid: (nk, dk) for ngr_short_range_tables."""
    nk, dk = C.c_uint32(), C.c_double()
    rc = lib().ngr_short_range_grid(C.c_double(r_s), C.c_double(r_cut), C.c_double(range_), C.byref(nk), C.byref(dk))
    if rc != 0:
        raise NgravsError(rc, "short_range_grid: bad arguments")
    return nk.value, dk.value


def short_range_tables(ctx: Context, *, phibar, f_full, r_s: float, r_cut: float, grid, dk: float) -> np.ndarray:
    """ngr_short_range_tables. phibar: host D x D x nk samples of k^2 phi(k)
    at k = m dk; f_full: host D x D x ntab full force factors at the table
    radii. Returns the D x D x ntab short-range tables (host)."""
    phibar = np.ascontiguousarray(phibar, dtype=np.float64)
    f_full = np.ascontiguousarray(f_full, dtype=np.float64)
    D, _, nk = phibar.shape
    ntab = f_full.shape[-1]
    out = np.empty((D, D, ntab))
    sp = ShortParams(D, ntab, GRIDS.get(grid, grid), nk, float(r_s), float(r_cut), float(dk))
    ctx._check(lib().ngr_short_range_tables(ctx.handle, C.byref(sp), _np(phibar), _np(f_full), _np(out)),
               "short-range tables")
    return out


class PmParams(C.Structure):
    _fields_ = [("N", C.c_uint32), ("D", C.c_uint32), ("box", C.c_double), ("r_s", C.c_double)]


class PmStats(C.Structure):
    _fields_ = [("ms_deposit", C.c_double), ("ms_fft_forward", C.c_double), ("ms_green", C.c_double),
                ("ms_fft_inverse", C.c_double), ("ms_interp", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


def pm_q_count(N: int) -> int:
    """Entries of a PM plan's phibar table per species pair: q = 0 .. 3 (N/2)^2."""
    return 3 * (N // 2) ** 2 + 1


class PM:
    """A PM plan (ngr_pm_create): N, D, box, r_s; host G (D x D) and phibar
    (D x D x pm_q_count(N), k^2 phi_ab(k) at |k| = 2 pi sqrt(q) / box)."""

    def __init__(self, ctx: Context, *, N: int, D: int, box: float, r_s: float, G, phibar):
        self.ctx = ctx
        G = np.ascontiguousarray(G, dtype=np.float64).reshape(D, D)
        phibar = np.ascontiguousarray(phibar, dtype=np.float64).reshape(D, D, pm_q_count(N))
        self._h = C.c_void_p()
        ctx._check(lib().ngr_pm_create(ctx.handle, C.byref(PmParams(N, D, float(box), float(r_s))), _np(G),
                                       _np(phibar), C.byref(self._h)), "pm create")

    def force(self, tree: Tree, acc, accumulate: bool = False) -> dict:
        """Long-range accelerations into the device tensor acc (3 x n, input order)."""
        st = PmStats()
        self.ctx._check(lib().ngr_pm_force(self.ctx.handle, self._h, tree.handle, C.c_void_p(_dev(acc)),
                                           int(bool(accumulate)), C.byref(st)), "pm force")
        return st.as_dict()

    def close(self):
        if self._h:
            self.ctx._check(lib().ngr_pm_destroy(self.ctx.handle, self._h), "pm destroy")
            self._h = None


class BatchBox:
    """One box of a batch: device tensors species (uint8, n), mass (float64,
    n), pos (float64, 3 x n) or lattice (uint64 lattice as int64, 3 x n), and
    acc (float64, 3 x n, written); host array G (D x D); tables (D x D x
    ntab) a host array, a float64 device tensor, or None; scalars as in
    tree_build / tree_force.
    group_size 0 lets the library choose."""

    def __init__(self, *, D, box, species, mass, acc, G, tables, grid, r_cut, eps, theta, pos=None, lattice=None,
                 leaf_size: int = 16, r_s: float = 0.0, group_size: int = 0, ntab: Optional[int] = None,
                 accumulator=None, eps_ab=None, relative=None, lattice_corr=None,
                 key_order: str = "morton"):
        self.n = int(species.shape[0])
        self.particles = Particles(self.n, D, float(box), _dev(pos), _dev(lattice), _dev(species), _dev(mass))
        self.tree = TreeParams(leaf_size, 0, KEY_ORDER[key_order])
        self.force = _force_params(D, G, tables, grid, r_s, r_cut, eps, theta, group_size, ntab, accumulator, eps_ab,
                                   relative, lattice_corr)
        self.acc = _dev(acc)
        self._keep = (species, mass, pos, lattice, acc)


def batch_build_force(ctx: Context, boxes, per_box: bool = False):
    """ngr_batch_build_force over a list of BatchBox. Returns the batch
    statistics as a dict, and with per_box=True also a list of per-box
    statistics dicts."""
    arr = (Box * len(boxes))()
    for k, b in enumerate(boxes):
        arr[k] = Box(b.particles, b.tree, b.force, b.acc)
    st = BatchStats()
    pb = (ForceStats * len(boxes))() if per_box else None
    ctx._check(lib().ngr_batch_build_force(ctx.handle, len(boxes), arr, C.byref(st), pb), "batch build and force")
    if per_box:
        return st.as_dict(), [pb[k].as_dict() for k in range(len(boxes))]
    return st.as_dict()


WAITING, ADMITTED, FINISHED = 0, 1, 2


class Server:
    """ngr_server_*: requests of leapfrog steps on many boxes, advanced
    together one force evaluation per tick (continuous batching)."""

    def __init__(self, ctx: Context, hbm_budget: int = 0, max_active: int = 0):
        self.ctx = ctx
        self._h = C.c_void_p()
        sp = ServerParams(int(hbm_budget), int(max_active))
        ctx._check(lib().ngr_server_create(ctx.handle, C.byref(sp), C.byref(self._h)), "server create")

    def submit(self, *, D, box, species, mass, G, tables, grid, r_cut, eps, theta, dt, steps, pos=None, lattice=None,
               vel=None, leaf_size: int = 16, r_s: float = 0.0, group_size: int = 0, ntab: Optional[int] = None,
               accumulator=None) -> int:
        """Device tensors species, mass, pos or lattice, vel (or None); host
        array G; tables a host array, a float64 device tensor or None. The
        data are copied; returns the request id."""
        n = int(species.shape[0])
        rq = RequestDesc(Particles(n, D, float(box), _dev(pos), _dev(lattice), _dev(species), _dev(mass)), _dev(vel),
                         TreeParams(leaf_size),
                         _force_params(D, G, tables, grid, r_s, r_cut, eps, theta, group_size, ntab, accumulator),
                         float(dt), int(steps))
        rid = C.c_uint64()
        self.ctx._check(lib().ngr_server_submit(self._h, C.byref(rq), C.byref(rid)), "server submit")
        return rid.value

    def tick(self) -> dict:
        st = TickStats()
        self.ctx._check(lib().ngr_server_tick(self._h, C.byref(st)), "server tick")
        return st.as_dict()

    def status(self, rid: int):
        state, evals = C.c_int(), C.c_uint32()
        self.ctx._check(lib().ngr_server_status(self._h, rid, C.byref(state), C.byref(evals)), "server status")
        return state.value, evals.value

    def take(self, rid: int, lattice=None, vel=None, acc=None):
        """Copy a finished request's lattice (uint64 as int64), velocities and
        accelerations (device tensors, 3 x n, any may be None) and release it."""
        self.ctx._check(lib().ngr_server_take(self._h, rid, C.c_void_p(_dev(lattice)), C.c_void_p(_dev(vel)),
                                              C.c_void_p(_dev(acc))), "server take")

    def close(self):
        if getattr(self, "_h", None):
            lib().ngr_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
