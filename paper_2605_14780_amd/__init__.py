"""Python binding of hipbc (``libhbc.so``, C ABI in ``include/hbc.h``).

Argument marshalling only: every step of the boundary-condition apply runs in
the library's HIP kernels.  Torch tensors supply device memory
(``data_ptr()``) and the current HIP stream; nothing here computes on them.
The binding raises if the library is not built; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhbc.so")

MAX_DIM = 6
OK, EINVAL, ERANGE, EOVERLAP, EALIAS, EUNCOVERED, ENOMEM, EHIP, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7, -8
F64, F32 = 0, 1
POINT_MAJOR, PLANE_MAJOR = 0, 1
STRICT_COVER, ALLOW_OVERLAP_SUM = 1, 2
PLAN_HOST_ONLY = 1
PLAN_NO_WINDOWS = 2
CS_SYNC, CS_LAGRANGE = 0, 1
OP_APPLY, OP_ADJOINT = 0, 1

SEG_ZERO, SEG_MAP, SEG_ELL, SEG_CSR, SEG_VEC, SEG_DATA_ROW = 0, 1, 2, 3, 4, 5


class HbcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hbc error {code}: {msg}")
        self.code = code


class Slice(C.Structure):
    _fields_ = [("start", C.c_int64), ("stop", C.c_int64), ("step", C.c_int64)]


class BoxT(C.Structure):
    _fields_ = [("lo", C.c_int64 * MAX_DIM), ("hi", C.c_int64 * MAX_DIM)]


class LayoutT(C.Structure):
    _fields_ = [("inner", C.c_int64), ("order", C.c_int32), ("vec_len", C.c_int32),
                ("vec_lo", C.c_int64), ("vec_stride", C.c_int64)]


class StatsT(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "ghost_cells", "rows_covered", "rows_uncovered", "rows_zero", "rows_map", "rows_ell", "rows_csr",
        "rows_vector_only", "rows_with_b", "nnz", "unique_sources", "segments", "tiles", "ghost_values")] + [
        ("alg_bytes", C.c_double), ("alg_bytes_adjoint", C.c_double), ("table_bytes", C.c_int64),
        ("rows_data", C.c_int64), ("rows_dead", C.c_int64), ("ghost_cells_live", C.c_int64),
        ("rows_wide", C.c_int64), ("wide_tiles", C.c_int64), ("rows_narrow", C.c_int64),
        ("rows_window", C.c_int64), ("window_runs", C.c_int64)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class TuneT(C.Structure):
    _fields_ = [("block", C.c_int32), ("lanes_per_row", C.c_int32), ("rows_per_tile", C.c_int32),
                ("persistent", C.c_int32), ("window_order", C.c_int32)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


P = C.c_void_p
I32, I64, U32, D = C.c_int32, C.c_int64, C.c_uint32, C.c_double
PI32, PI64, PD = C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_double)

# name -> (restype, argtypes); the full C ABI
SIGNATURES = {
    "hbc_last_error": (C.c_char_p, []),
    "hbc_grid_create": (I32, [I32, PI64, PI64, C.POINTER(P)]),
    "hbc_grid_add_block": (I32, [P, C.POINTER(Slice), C.POINTER(Slice), PI32]),
    "hbc_grid_cells": (I64, [P]),
    "hbc_grid_block_cells": (I32, [P, I32, PI64, PI64]),
    "hbc_grid_destroy": (None, [P]),
    "hbc_cs_grid_create": (I32, [I64, I64, C.POINTER(P)]),
    "hbc_cart_grid_create": (I32, [PI32, PI64, I64, C.POINTER(P)]),
    "hbc_program_create": (I32, [P, C.POINTER(P)]),
    "hbc_program_destroy": (None, [P]),
    "hbc_program_set_flags": (I32, [P, U32]),
    "hbc_program_add_map": (I32, [P, C.POINTER(BoxT), PI64, PI64, D, PI32, PI32]),
    "hbc_program_add_zero": (I32, [P, C.POINTER(BoxT), PI32]),
    "hbc_program_add_zero_rest": (I32, [P, I32, PI32]),
    "hbc_program_add_ell": (I32, [P, C.POINTER(BoxT), I32, PI64, PD, PI32, PI32]),
    "hbc_program_add_csr": (I32, [P, C.POINTER(BoxT), PI64, PI64, PD, PI32, PI32]),
    "hbc_program_add_vector": (I32, [P, C.POINTER(BoxT), I64, PD, PI32]),
    "hbc_program_set_consumer": (I32, [P, I32, PI64]),
    "hbc_program_add_data_csr": (I32, [P, C.POINTER(BoxT), PI64, PI64, PD, PI32]),
    "hbc_cs_program_add_edge_average": (I32, [P, I64]),
    "hbc_cs_program_add_quadrature": (I32, [P, I64, I64, I32, I32]),
    "hbc_cs_program_add": (I32, [P, I64, I64, I32, I32, PI32, PD]),
    "hbc_cart_program_add_halo": (I32, [P, PI32, PI64, I64, I32]),
    "hbc_plan_create": (I32, [P, C.POINTER(LayoutT), I32, U32, C.POINTER(P)]),
    "hbc_plan_destroy": (None, [P]),
    "hbc_plan_stats": (I32, [P, C.POINTER(StatsT)]),
    "hbc_plan_row": (I32, [P, I64, I64, I32, PI64, PD, PI32, PD, PI32, PI32]),
    "hbc_plan_set_vector": (I32, [P, I32, PD, P]),
    "hbc_plan_get_tune": (I32, [P, C.POINTER(TuneT)]),
    "hbc_plan_set_tune": (I32, [P, C.POINTER(TuneT)]),
    "hbc_plan_autotune": (I32, [P, C.POINTER(P), I64, I32, C.c_char_p, P, PD]),
    "hbc_apply": (I32, [P, P, I64, P]),
    "hbc_apply_adjoint": (I32, [P, P, I64, P]),
    "hbc_apply_adjoint_noalloc": (I32, [P, P, I64, P]),
    "hbc_plan_kernels": (I32, [P, I32, C.c_char_p, I64, PI64]),
    "hbc_program_box_rows": (I32, [P, C.POINTER(BoxT), PI64]),
    "hbc_consumer_create": (I32, [P, I32, PI64, PD, C.POINTER(P)]),
    "hbc_consumer_apply": (I32, [P, P, I64, P, I64, I32, P]),
    "hbc_consumer_stats": (I32, [P, PI64, PI64]),
    "hbc_consumer_destroy": (None, [P]),
    "hbc_time_apply": (I32, [P, C.POINTER(P), I64, I32, I32, P, PD]),
    "hbc_graph_create": (I32, [P, I32, C.POINTER(P), I64, I32, I32, P, C.POINTER(P)]),
    "hbc_graph_launch": (I32, [P, P]),
    "hbc_graph_destroy": (None, [P]),
    "hbc_stencil27": (I32, [P, P, I64, P, I64, P]),
    "hbc_fused_stencil27": (I32, [P, P, I64, P, I64, I32, P]),
    "hbc_cs_lagrange_weights": (I32, [I64, I64, P, P, P]),
    "hbc_batch_create": (I32, [C.POINTER(P), I32, C.POINTER(P)]),
    "hbc_batch_destroy": (None, [P]),
    "hbc_batch_bind": (I32, [P, C.POINTER(P), PI64]),
    "hbc_batch_apply": (I32, [P, P]),
    "hbc_batch_graph_capture": (I32, [P, P]),
    "hbc_batch_graph_launch": (I32, [P, P]),
    "hbc_batch_get_tune": (I32, [P, C.POINTER(TuneT)]),
    "hbc_batch_set_tune": (I32, [P, C.POINTER(TuneT)]),
    "hbc_batch_autotune": (I32, [P, C.c_char_p, P, PD]),
    "hbc_batch_stats": (I32, [P, C.POINTER(StatsT)]),
}

_lib = None


def lib():
    """Load libhbc.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                               "or python -m paper_2605_14780_amd.build")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != OK:
        raise HbcError(rc, lib().hbc_last_error().decode())


def _i64(seq):
    a = np.ascontiguousarray(np.asarray(seq, dtype=np.int64))
    return a, a.ctypes.data_as(PI64)


def _f64(seq):
    a = np.ascontiguousarray(np.asarray(seq, dtype=np.float64))
    return a, a.ctypes.data_as(PD)


def _box(rows):
    b = BoxT()
    for d, (lo, hi) in enumerate(rows):
        b.lo[d], b.hi[d] = int(lo), int(hi)
    return b


def _rot(rot):
    if rot is None:
        return None, None
    a = np.ascontiguousarray(np.asarray(rot, dtype=np.int32).reshape(4))
    return a, a.ctypes.data_as(PI32)


def _stream(stream):
    if stream is not None:
        return P(int(stream))
    import torch
    return P(int(torch.cuda.current_stream().cuda_stream))


# ---- grid ------------------------------------------------------------------------------
class Grid:
    def __init__(self, lo=None, hi=None, _handle=None):
        self._h = P()
        if _handle is not None:
            self._h = _handle
        else:
            lo_a, lo_p = _i64(lo)
            hi_a, hi_p = _i64(hi)
            _check(lib().hbc_grid_create(len(lo_a), lo_p, hi_p, C.byref(self._h)))
        self.ndim = None

    @classmethod
    def cubed_sphere(cls, N, h):
        g = P()
        _check(lib().hbc_cs_grid_create(N, h, C.byref(g)))
        return cls(_handle=g)

    @classmethod
    def cartesian(cls, nb, n, h):
        nb_a = np.ascontiguousarray(np.asarray(nb, dtype=np.int32))
        n_a, n_p = _i64(n)
        g = P()
        _check(lib().hbc_cart_grid_create(nb_a.ctypes.data_as(PI32), n_p, h, C.byref(g)))
        return cls(_handle=g)

    def add_block(self, full, data):
        """full / data: per dimension (start, stop) or (start, stop, step)."""
        nd = len(full)
        F = (Slice * nd)(*[Slice(s[0], s[1], s[2] if len(s) > 2 else 1) for s in full])
        Dd = (Slice * nd)(*[Slice(s[0], s[1], s[2] if len(s) > 2 else 1) for s in data])
        bid = I32()
        _check(lib().hbc_grid_add_block(self._h, F, Dd, C.byref(bid)))
        return bid.value

    @property
    def cells(self):
        return int(lib().hbc_grid_cells(self._h))

    def block_cells(self, b):
        first, n = I64(), I64()
        _check(lib().hbc_grid_block_cells(self._h, b, C.byref(first), C.byref(n)))
        return first.value, n.value

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hbc_grid_destroy(self._h)
            self._h = None


# ---- program ---------------------------------------------------------------------------
class Program:
    def __init__(self, grid: Grid):
        self._h = P()
        self.grid = grid
        self._vec_len = {}  # sub-vector id -> number of values it takes
        _check(lib().hbc_program_create(grid._h, C.byref(self._h)))

    def box_rows(self, rows):
        """Rows (grid points) the row box selects."""
        n = I64()
        _check(lib().hbc_program_box_rows(self._h, C.byref(_box(rows)), C.byref(n)))
        return n.value

    def _need(self, what, got, want):
        if got != want:
            raise ValueError(f"{what}: {got} values given, the row box needs {want}")

    def set_flags(self, flags):
        _check(lib().hbc_program_set_flags(self._h, flags))

    def add_map(self, rows, M, offset, weight=1.0, rot=None):
        M_a, M_p = _i64(np.asarray(M).reshape(-1))
        o_a, o_p = _i64(offset)
        self._need("M", len(M_a), len(rows) ** 2)
        self._need("offset", len(o_a), len(rows))
        r_a, r_p = _rot(rot)
        sid = I32()
        _check(lib().hbc_program_add_map(self._h, C.byref(_box(rows)), M_p, o_p, float(weight), r_p, C.byref(sid)))
        return sid.value

    def add_zero(self, rows):
        sid = I32()
        _check(lib().hbc_program_add_zero(self._h, C.byref(_box(rows)), C.byref(sid)))
        return sid.value

    def add_zero_rest(self, block):
        sid = I32()
        _check(lib().hbc_program_add_zero_rest(self._h, block, C.byref(sid)))
        return sid.value

    def add_ell(self, rows, width, cols, vals, rot=None):
        c_a, c_p = _i64(np.asarray(cols).reshape(-1))
        v_a, v_p = _f64(np.asarray(vals).reshape(-1))
        n = self.box_rows(rows) * width
        self._need("cols", len(c_a), n)
        self._need("vals", len(v_a), n)
        r_a, r_p = _rot(rot)
        sid = I32()
        _check(lib().hbc_program_add_ell(self._h, C.byref(_box(rows)), width, c_p, v_p, r_p, C.byref(sid)))
        return sid.value

    def add_csr(self, rows, row_ptr, cols, vals, rot=None):
        p_a, p_p = _i64(row_ptr)
        c_a, c_p = _i64(np.asarray(cols).reshape(-1))
        v_a, v_p = _f64(np.asarray(vals).reshape(-1))
        self._check_csr(rows, p_a, c_a, v_a)
        r_a, r_p = _rot(rot)
        sid = I32()
        _check(lib().hbc_program_add_csr(self._h, C.byref(_box(rows)), p_p, c_p, v_p, r_p, C.byref(sid)))
        return sid.value

    def _check_csr(self, rows, p_a, c_a, v_a):
        self._need("row_ptr", len(p_a), self.box_rows(rows) + 1)
        self._need("cols", len(c_a), int(p_a[-1]))
        self._need("vals", len(v_a), int(p_a[-1]))

    def add_vector(self, rows, values, ninner=1):
        v_a, v_p = _f64(np.asarray(values).reshape(-1))
        n = self.box_rows(rows) * ninner
        self._need("values", len(v_a), n)
        sid = I32()
        _check(lib().hbc_program_add_vector(self._h, C.byref(_box(rows)), ninner, v_p, C.byref(sid)))
        self._vec_len[sid.value] = n
        return sid.value

    def set_consumer(self, offsets):
        """Read offsets of the consuming operator (n x ndim); ghost rows no read reaches are dropped."""
        o = np.asarray(offsets, dtype=np.int64).reshape(-1)
        o_a, o_p = _i64(o)
        n = 0 if o.size == 0 else len(offsets)
        _check(lib().hbc_program_set_consumer(self._h, n, o_p if n else None))

    def add_data_csr(self, rows, row_ptr, cols, vals):
        """Rows on data cells (block-edge averaging); every row reads the input field."""
        p_a, p_p = _i64(row_ptr)
        c_a, c_p = _i64(np.asarray(cols).reshape(-1))
        v_a, v_p = _f64(np.asarray(vals).reshape(-1))
        self._check_csr(rows, p_a, c_a, v_a)
        sid = I32()
        _check(lib().hbc_program_add_data_csr(self._h, C.byref(_box(rows)), p_p, c_p, v_p, C.byref(sid)))
        return sid.value

    def cs_add_quadrature(self, N, h, q=2, vector=False):
        """Wide rows: Gauss average over each ghost cell of cubic tensor-product reconstructions."""
        _check(lib().hbc_cs_program_add_quadrature(self._h, N, h, q, int(bool(vector))))

    def cs_add_edge_average(self, Np):
        """Averaging of co-located face-boundary points of a vertex-centred cubed sphere."""
        _check(lib().hbc_cs_program_add_edge_average(self._h, Np))

    def cs_add(self, N, h, mode, vector=False, base=None, w=None):
        if base is None:
            b_a, b_p, w_a, w_p = None, None, None, None
        else:
            b_a = np.ascontiguousarray(np.asarray(base, dtype=np.int32).reshape(-1))
            b_p = b_a.ctypes.data_as(PI32)
            w_a, w_p = _f64(np.asarray(w).reshape(-1))
            if len(b_a) != h * N or len(w_a) != 4 * h * N:
                raise ValueError(f"base / w: {len(b_a)} / {len(w_a)} values given, {h * N} / {4 * h * N} needed")
        _check(lib().hbc_cs_program_add(self._h, N, h, mode, int(bool(vector)), b_p, w_p))

    def cart_add_halo(self, nb, n, h, periodic=0):
        nb_a = np.ascontiguousarray(np.asarray(nb, dtype=np.int32))
        n_a, n_p = _i64(n)
        if len(nb_a) != 3 or len(n_a) != 3:
            raise ValueError("nb and n take 3 values each (z, y, x)")
        _check(lib().hbc_cart_program_add_halo(self._h, nb_a.ctypes.data_as(PI32), n_p, h, periodic))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hbc_program_destroy(self._h)
            self._h = None


# ---- plan ------------------------------------------------------------------------------
class Plan:
    def __init__(self, program: Program, inner=1, order=POINT_MAJOR, vec=None, dtype=F64, host_only=False,
                 windows=True):
        """vec = (lo, stride, len) of the two vector components' inner slots, or None;
        windows=False serves sliding-window rows with the general row kernel."""
        self._h = P()
        lay = LayoutT()
        lay.inner = inner
        lay.order = order
        if vec is not None:
            lay.vec_lo, lay.vec_stride, lay.vec_len = vec
        flags = (PLAN_HOST_ONLY if host_only else 0) | (0 if windows else PLAN_NO_WINDOWS)
        _check(lib().hbc_plan_create(program._h, C.byref(lay), dtype, flags, C.byref(self._h)))
        self._vec_len = dict(program._vec_len)
        self.inner = inner
        self.order = order
        self.dtype = dtype
        self.host_only = host_only
        self.ncells = program.grid.cells
        self.nelem = self.ncells * inner

    def stats(self):
        s = StatsT()
        _check(lib().hbc_plan_stats(self._h, C.byref(s)))
        return s.as_dict()

    def row(self, cell, l=0, cap=64):
        cols = (C.c_int64 * cap)()
        vals = (C.c_double * cap)()
        nnz, kind, rot = I32(), I32(), I32()
        b = D()
        _check(lib().hbc_plan_row(self._h, cell, l, cap, cols, vals, C.byref(nnz), C.byref(b), C.byref(kind),
                                  C.byref(rot)))
        n = min(nnz.value, cap)
        return kind.value, list(cols[:n]), list(vals[:n]), b.value, rot.value

    def set_vector(self, sub_id, values, stream=None):
        """New values for sub-vector sub_id, laid out as for Program.add_vector."""
        v_a, v_p = _f64(np.asarray(values).reshape(-1))
        # an id that is no sub-vector is refused by the library before it reads values
        if sub_id in self._vec_len and len(v_a) != self._vec_len[sub_id]:
            raise ValueError(f"values: {len(v_a)} given, sub-vector {sub_id} takes {self._vec_len[sub_id]}")
        st = P(0) if self.host_only else _stream(stream)
        _check(lib().hbc_plan_set_vector(self._h, sub_id, v_p, st))

    def kernels(self, op=None):
        """Demangled names of the kernels one apply (or adjoint, op=OP_ADJOINT) launches."""
        op = OP_APPLY if op is None else op
        n = I64()
        _check(lib().hbc_plan_kernels(self._h, op, None, 0, C.byref(n)))
        buf = C.create_string_buffer(n.value + 1)
        _check(lib().hbc_plan_kernels(self._h, op, buf, n.value + 1, C.byref(n)))
        return [x for x in buf.value.decode().split("\n") if x]

    @property
    def tune(self):
        t = TuneT()
        _check(lib().hbc_plan_get_tune(self._h, C.byref(t)))
        return t.as_dict()

    @tune.setter
    def tune(self, d):
        t = TuneT(**d)
        _check(lib().hbc_plan_set_tune(self._h, C.byref(t)))

    def autotune(self, fields, cache_path=None, stream=None):
        """Pick the fastest launch shape on ``fields`` (ghosts overwritten); returns ms per apply."""
        ptrs = [_field(self, f) for f in fields]
        arr = (P * len(ptrs))(*[p for p, _ in ptrs])
        ms = D()
        _check(lib().hbc_plan_autotune(self._h, arr, ptrs[0][1], len(ptrs),
                                       cache_path.encode() if cache_path else None, _stream(stream), C.byref(ms)))
        return ms.value

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hbc_plan_destroy(self._h)
            self._h = None


def _field(plan: Plan, t):
    import torch
    want = torch.float64 if plan.dtype == F64 else torch.float32
    if not t.is_cuda or t.dtype != want or not t.is_contiguous():
        raise ValueError(f"field must be a contiguous {want} tensor on the GPU")
    return P(t.data_ptr()), int(t.numel())


def apply(plan: Plan, field, stream=None):
    """ghosts := A x + b, in place on ``field`` (the library's apply kernel)."""
    ptr, n = _field(plan, field)
    _check(lib().hbc_apply(plan._h, ptr, n, _stream(stream)))
    return field


def apply_adjoint(plan: Plan, grad, stream=None):
    """In place: data += A^T (covered ghost part), covered ghosts := 0."""
    ptr, n = _field(plan, grad)
    _check(lib().hbc_apply_adjoint(plan._h, ptr, n, _stream(stream)))
    return grad


def apply_adjoint_noalloc(plan: Plan, grad, stream=None):
    """As apply_adjoint, allocating nothing (the library's static counter array)."""
    ptr, n = _field(plan, grad)
    _check(lib().hbc_apply_adjoint_noalloc(plan._h, ptr, n, _stream(stream)))
    return grad


def time_apply(plan: Plan, fields, reps, stream=None):
    """Mean ms per apply of ``reps`` applies (cycling over ``fields``) in one HIP graph."""
    ptrs = [_field(plan, f) for f in fields]
    arr = (P * len(ptrs))(*[p for p, _ in ptrs])
    ms = D()
    _check(lib().hbc_time_apply(plan._h, arr, ptrs[0][1], len(ptrs), reps, _stream(stream), C.byref(ms)))
    return ms.value


class ApplyGraph:
    """``reps`` applies (or adjoints) of ``plan`` over ``fields`` (cycled) captured in one HIP graph."""

    def __init__(self, plan: Plan, fields, reps, stream=None, op=OP_APPLY):
        ptrs = [_field(plan, f) for f in fields]
        arr = (P * len(ptrs))(*[p for p, _ in ptrs])
        self._h = P()
        self._fields = list(fields)  # keep the memory alive with the graph
        self.reps = reps
        _check(lib().hbc_graph_create(plan._h, op, arr, ptrs[0][1], len(ptrs), reps, _stream(stream),
                                      C.byref(self._h)))

    def launch(self, stream=None):
        _check(lib().hbc_graph_launch(self._h, _stream(stream)))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hbc_graph_destroy(self._h)
            self._h = None


class Consumer:
    """A stencil (offsets, weights) reading the plan's field after the BC; apply(x, y, fused)."""

    def __init__(self, plan: Plan, offsets, weights):
        o = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        if o.ndim != 2:
            raise ValueError("offsets: (noffsets, ndim)")
        w_a, w_p = _f64(np.asarray(weights, dtype=np.float64).reshape(-1))
        if len(w_a) != o.shape[0]:
            raise ValueError("one weight per offset")
        self._h = P()
        self.plan = plan  # the library keeps a pointer to the plan
        _check(lib().hbc_consumer_create(plan._h, o.shape[0], o.ctypes.data_as(PI64), w_p, C.byref(self._h)))

    def stats(self):
        r, e = I64(), I64()
        _check(lib().hbc_consumer_stats(self._h, C.byref(r), C.byref(e)))
        return {"boundary_rows": r.value, "boundary_entries": e.value}

    def apply(self, x, y, fused=True, stream=None):
        xp, xn = _field(self.plan, x)
        if y.dtype != x.dtype or not y.is_contiguous() or not y.is_cuda:
            raise ValueError("y must be a contiguous GPU tensor of x's dtype")
        _check(lib().hbc_consumer_apply(self._h, xp, xn, P(y.data_ptr()), int(y.numel()), int(bool(fused)),
                                        _stream(stream)))
        return y

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hbc_consumer_destroy(self._h)
            self._h = None


def stencil27(plan: Plan, x, y, stream=None):
    xp, xn = _field(plan, x)
    yp, yn = P(y.data_ptr()), int(y.numel())
    if y.dtype != x.dtype or not y.is_contiguous() or not y.is_cuda:
        raise ValueError("y must be a contiguous GPU tensor of x's dtype")
    _check(lib().hbc_stencil27(plan._h, xp, xn, yp, yn, _stream(stream)))
    return y


def fused_stencil27(plan: Plan, x, y, write_ghosts=True, stream=None):
    xp, xn = _field(plan, x)
    yp, yn = P(y.data_ptr()), int(y.numel())
    if y.dtype != x.dtype or not y.is_contiguous() or not y.is_cuda:
        raise ValueError("y must be a contiguous GPU tensor of x's dtype")
    _check(lib().hbc_fused_stencil27(plan._h, xp, xn, yp, yn, int(bool(write_ghosts)), _stream(stream)))
    return y


def cs_lagrange_weights(N, h, stream=None):
    """FP64 Lagrange bases and weights on the device: (base int32 [h*N], w float64 [h*N, 4])."""
    import torch
    base = torch.empty(h * N, dtype=torch.int32, device="cuda")
    w = torch.empty(h * N, 4, dtype=torch.float64, device="cuda")
    _check(lib().hbc_cs_lagrange_weights(N, h, P(base.data_ptr()), P(w.data_ptr()), _stream(stream)))
    return base, w


def cs_program(N, h, mode=CS_LAGRANGE, vector=False, stream=None):
    """Grid + program of the cubed-sphere BC; Lagrange weights are built on the GPU."""
    g = Grid.cubed_sphere(N, h)
    p = Program(g)
    if mode == CS_LAGRANGE:
        import torch
        base, w = cs_lagrange_weights(N, h, stream)
        torch.cuda.synchronize()
        p.cs_add(N, h, mode, vector, base.cpu().numpy(), w.cpu().numpy())
    else:
        p.cs_add(N, h, mode, vector)
    return g, p


# ---- batch -----------------------------------------------------------------------------
class Batch:
    def __init__(self, plans):
        self.plans = list(plans)
        arr = (P * len(self.plans))(*[p._h for p in self.plans])
        self._h = P()
        _check(lib().hbc_batch_create(arr, len(self.plans), C.byref(self._h)))

    def bind(self, fields):
        ptrs = [_field(p, f) for p, f in zip(self.plans, fields)]
        arr = (P * len(ptrs))(*[q for q, _ in ptrs])
        n_a, n_p = _i64([n for _, n in ptrs])
        _check(lib().hbc_batch_bind(self._h, arr, n_p))
        self._fields = list(fields)

    def apply(self, stream=None):
        _check(lib().hbc_batch_apply(self._h, _stream(stream)))

    def graph_capture(self, stream=None):
        _check(lib().hbc_batch_graph_capture(self._h, _stream(stream)))

    def graph_launch(self, stream=None):
        _check(lib().hbc_batch_graph_launch(self._h, _stream(stream)))

    def autotune(self, cache_path=None, stream=None):
        ms = D()
        _check(lib().hbc_batch_autotune(self._h, cache_path.encode() if cache_path else None, _stream(stream),
                                        C.byref(ms)))
        return ms.value

    @property
    def tune(self):
        t = TuneT()
        _check(lib().hbc_batch_get_tune(self._h, C.byref(t)))
        return t.as_dict()

    @tune.setter
    def tune(self, d):
        t = TuneT(**d)
        _check(lib().hbc_batch_set_tune(self._h, C.byref(t)))

    def stats(self):
        s = StatsT()
        _check(lib().hbc_batch_stats(self._h, C.byref(s)))
        return s.as_dict()

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hbc_batch_destroy(self._h)
            self._h = None


# ---- autograd ----------------------------------------------------------------------------
def _autograd():
    import torch

    class BCApply(torch.autograd.Function):
        """u -> u' with covered ghosts := A x + b (forward on a copy); backward = hbc_apply_adjoint."""

        @staticmethod
        def forward(ctx, plan, u):
            ctx.plan = plan
            out = u.detach().clone()
            apply(plan, out)
            return out

        @staticmethod
        def backward(ctx, g):
            gu = g.detach().contiguous().clone()
            apply_adjoint(ctx.plan, gu)
            return None, gu

    return BCApply


_BCApply = None


def bc_apply(plan: Plan, u):
    """Differentiable apply (torch.autograd.Function)."""
    global _BCApply
    if _BCApply is None:
        _BCApply = _autograd()
    return _BCApply.apply(plan, u)
