"""Thin Python binding of libpagefem.so (ctypes).

Argument marshalling only: every function forwards torch tensors' device pointers, sizes
and the current HIP stream to the C entry point of the same name (without the ``pf_``
prefix) declared in ``include/pagefem.h``.  PyTorch supplies device memory and streams;
all computation happens in the library's HIP kernels.  There is no CPU fallback: if the
library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpagefem.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2404_16039_amd.build`")

_lib = C.CDLL(LIB_PATH)

F32, F64 = 0, 1
STATUS = {0: "PF_OK", 1: "PF_EINVAL", 2: "PF_EDTYPE", 3: "PF_EORDER", 4: "PF_ENOMEM", 5: "PF_EHIP",
          6: "PF_EINDEX", 7: "PF_ELIMIT", 8: "PF_EBUDGET", 9: "PF_ESTATE"}


class PagefemError(RuntimeError):
    def __init__(self, name, code, msg):
        super().__init__(f"{name}: {STATUS.get(code, code)}: {msg}")
        self.code = code


class Pages(C.Structure):
    """pf_pages: page shape, count and element strides (s_page = 0 broadcasts)."""
    _fields_ = [("rows", C.c_int32), ("cols", C.c_int32), ("count", C.c_int64),
                ("s_row", C.c_int64), ("s_col", C.c_int64), ("s_page", C.c_int64)]


class Fallback(C.Structure):
    """pf_fallback: FP64 routing thresholds of the FP32 path."""
    _fields_ = [("tau_abs", C.c_double), ("tau_cond", C.c_double), ("enable", C.c_int32)]


def pages(count, rows, cols):
    """Descriptor of the paper's layout: column-major pages stored back to back."""
    return Pages(rows, cols, count, 1, rows, rows * cols)


def pages_soa(count, rows, cols):
    """Descriptor of the structure-of-arrays layout: component (r, c) of all pages contiguous."""
    return Pages(rows, cols, count, count, rows * count, 1)


def pages_bcast(rows, cols, count=1):
    """One column-major page broadcast to every index."""
    return Pages(rows, cols, count, 1, rows, 0)


class Group(C.Structure):
    _fields_ = [("order", C.c_int32), ("ops", C.c_int32), ("count", C.c_int64), ("a", C.c_void_p),
                ("b", C.c_void_p), ("x", C.c_void_p), ("c", C.c_void_p), ("det", C.c_void_p)]


class OrderSchedule(C.Structure):
    _fields_ = [("lanes", C.c_int32), ("staged", C.c_int32), ("tile", C.c_int32)]


class Schedule(C.Structure):
    _fields_ = [("waves", C.c_int32), ("order", OrderSchedule * 5)]

    def as_dict(self):
        return {"waves": self.waves,
                "order": {n: (self.order[n].lanes, self.order[n].staged, self.order[n].tile) for n in range(1, 5)}}


class Job(C.Structure):
    _fields_ = [("dim", C.c_int32), ("prec", C.c_int32), ("nn", C.c_int64), ("ne", C.c_int64),
                ("coords", C.c_void_p), ("elems", C.c_void_p), ("topology", C.c_uint64), ("arrival", C.c_double),
                ("fb", Fallback), ("valsK", C.c_void_p), ("valsM", C.c_void_p), ("vals_cap", C.c_int64),
                ("kind", C.c_int32), ("order", C.c_int32), ("ops", C.c_int32), ("reserved", C.c_int32),
                ("count", C.c_int64), ("a", C.c_void_p), ("b", C.c_void_p), ("x", C.c_void_p), ("c", C.c_void_p),
                ("det", C.c_void_p)]


class JobResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("done", C.c_int32), ("nnz", C.c_int64), ("routed", C.c_int64),
                ("arrival", C.c_double), ("admitted", C.c_double), ("finished", C.c_double),
                ("copied", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64), ("elements", C.c_int64),
                ("ticks", C.c_int64), ("launches", C.c_int64), ("max_batch", C.c_int64),
                ("cache_hits", C.c_int64), ("cache_misses", C.c_int64), ("evictions", C.c_int64),
                ("latency_p50", C.c_double), ("latency_p99", C.c_double), ("latency_mean", C.c_double),
                ("latency_max", C.c_double), ("first_arrival", C.c_double), ("last_finish", C.c_double),
                ("jobs_per_s", C.c_double), ("elements_per_s", C.c_double), ("hbm_in_use", C.c_int64),
                ("hbm_high_water", C.c_int64), ("pages", C.c_int64), ("pages_per_s", C.c_double),
                ("evict_s", C.c_double), ("build_start_s", C.c_double), ("tick_s", C.c_double),
                ("admit_waits", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


SERVER_NOFUSE, SERVER_NOCACHE = 1, 2
JOB_ASSEMBLY, JOB_PAGES = 0, 1
OP_INV, OP_MTIMES = 1, 2
TUNE_CACHED, TUNE_FORCE, TUNE_DEFAULT = 0, 1, 2


def fallback(tau_abs=0.0, tau_cond=1e6, enable=True):
    return Fallback(float(tau_abs), float(tau_cond), 1 if enable else 0)


P = C.c_void_p
I32 = C.c_int
I64 = C.c_int64
PP = C.POINTER(Pages)
FP = C.POINTER(Fallback)

_sig = {
    "pf_last_error": ([], C.c_char_p),
    "pf_version": ([], C.c_int),
    "pf_page_det": ([I32, PP, P, P, FP, P, P, P], C.c_int),
    "pf_page_inv": ([I32, PP, P, PP, P, P, FP, P, P, P], C.c_int),
    "pf_page_transpose": ([I32, PP, P, PP, P, P], C.c_int),
    "pf_page_mtimes": ([I32, PP, P, I32, PP, P, I32, PP, P, P], C.c_int),
    "pf_page_mv": ([I32, PP, P, I32, PP, P, PP, P, P], C.c_int),
    "pf_page_scale": ([I32, P, I64, PP, P, PP, P, P], C.c_int),
    "pf_page_bilinear": ([I32, PP, P, PP, P, PP, P, P, P], C.c_int),
    "pf_elem_geometry": ([I32, I32, I64, P, I64, P, P, P, P, P, P, FP, P, P, P], C.c_int),
    "pf_elem_stiffness_mass": ([I32, I32, I64, P, I64, P, P, P, P, P, FP, P, P, P], C.c_int),
    "pf_boundary_normals": ([I32, I32, I64, P, I64, P, P, P, P], C.c_int),
    "pf_quad_points": ([I32, I32, I64, P, I64, P, P, P], C.c_int),
    "pf_assemble_quad": ([P, I32, P, I32, P, P, P, P, FP, P, P], C.c_int),
    "pf_csr_faces": ([P, P, P, P], C.c_int),
    "pf_csr_faces_info": ([P, C.POINTER(I64), C.POINTER(I64), C.POINTER(P), C.POINTER(P), C.POINTER(P),
                           C.POINTER(P)], C.c_int),
    "pf_simplex_points": ([I32, I32, I64, P, I64, P, I32, P, P, P], C.c_int),
    "pf_p2_elements": ([I32, I32, I64, P, I64, P, I32, P, P, P, I32, P, P, P, P, P, FP, P, P], C.c_int),
    "pf_gi": ([I32, I64, I32, I32, P, P, P, P, P, P, P], C.c_int),
    "pf_rhs": ([P, I32, P, P, I32, P, P, P, FP, P, P], C.c_int),
    "pf_energies": ([P, I32, P, P, I32, P, P, P, P, P, P, FP, P, P], C.c_int),
    "pf_energies_noalloc": ([P, I32, P, P, I32, P, P, P, P, P, P, FP, P, P], C.c_int),
    "pf_csr_create": ([C.POINTER(P)], C.c_int),
    "pf_csr_symbolic": ([P, I32, I64, I64, P, P], C.c_int),
    "pf_csr_symbolic_p2": ([P, I32, I64, I64, P, P], C.c_int),
    "pf_csr_assemble_pages": ([P, I32, P, P, P, P, P], C.c_int),
    "pf_csr_info": ([P, C.POINTER(I64), C.POINTER(I64), C.POINTER(P), C.POINTER(P)], C.c_int),
    "pf_csr_numeric_info": ([P, I32, C.POINTER(I32), C.POINTER(I32)], C.c_int),
    "pf_csr_memory": ([P, C.POINTER(I64), C.POINTER(I64)], C.c_int),
    "pf_csr_set_timing": ([P, C.c_int], C.c_int),
    "pf_csr_stage_times": ([P, C.POINTER(C.c_double), C.POINTER(I64)], C.c_int),
    "pf_assemble": ([P, I32, P, P, P, P, P, P, FP, P, P], C.c_int),
    "pf_csr_destroy": ([P], None),
    "pf_plan_create": ([I32, I32, FP, C.POINTER(P)], C.c_int),
    "pf_plan_set_groups": ([P, C.POINTER(Group), I32], C.c_int),
    "pf_plan_get_schedule": ([P, C.POINTER(Schedule)], C.c_int),
    "pf_plan_set_schedule": ([P, C.POINTER(Schedule)], C.c_int),
    "pf_plan_tune": ([P, C.c_char_p, I32, P], C.c_int),
    "pf_plan_run": ([P, P, P], C.c_int),
    "pf_plan_launch": ([P, P, P], C.c_int),
    "pf_plan_info": ([P, C.POINTER(I64), C.POINTER(I32), C.POINTER(I32)], C.c_int),
    "pf_plan_destroy": ([P], None),
    "pf_server_create": ([C.c_size_t, I32, I32, C.POINTER(P)], C.c_int),
    "pf_server_now": ([P], C.c_double),
    "pf_server_submit": ([P, C.POINTER(Job), C.POINTER(C.c_uint64)], C.c_int),
    "pf_server_footprint": ([C.POINTER(Job), C.POINTER(C.c_size_t)], C.c_int),
    "pf_server_poll": ([P, C.c_uint64, C.POINTER(JobResult)], C.c_int),
    "pf_server_wait": ([P, C.c_uint64, C.POINTER(JobResult)], C.c_int),
    "pf_server_drain": ([P], C.c_int),
    "pf_server_stats": ([P, C.POINTER(Stats)], C.c_int),
    "pf_server_destroy": ([P], None),
}
for _name, (_args, _res) in _sig.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res


def exported_symbols():
    return sorted(_sig)


def last_error() -> str:
    return _lib.pf_last_error().decode()


def version() -> int:
    return _lib.pf_version()


def _chk(rc, name):
    if rc != 0:
        raise PagefemError(name, rc, last_error())


def _p(t):
    if t is None:
        return None
    if isinstance(t, int):
        return P(t)
    if not t.is_cuda:
        raise ValueError("pagefem tensors must live in device memory")
    return P(t.data_ptr())


def _s(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return P(s.cuda_stream)


def _dt(t):
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise ValueError(f"unsupported dtype {t.dtype}")


def _ref(x, typ):
    return None if x is None else C.byref(x)


# ----------------------------------------------------------------------------- page ops
def page_det(A: Pages, a, det, fb=None, flags=None, counters=None, stream=None):
    _chk(_lib.pf_page_det(_dt(a), C.byref(A), _p(a), _p(det), _ref(fb, Fallback), _p(flags), _p(counters),
                          _s(stream)), "pf_page_det")


def page_inv(A: Pages, a, X: Pages, x, det=None, fb=None, flags=None, counters=None, stream=None):
    _chk(_lib.pf_page_inv(_dt(a), C.byref(A), _p(a), C.byref(X), _p(x), _p(det), _ref(fb, Fallback), _p(flags),
                          _p(counters), _s(stream)), "pf_page_inv")


def page_transpose(A: Pages, a, T: Pages, t, stream=None):
    _chk(_lib.pf_page_transpose(_dt(a), C.byref(A), _p(a), C.byref(T), _p(t), _s(stream)), "pf_page_transpose")


def page_mtimes(A: Pages, a, transA, B: Pages, b, transB, Cd: Pages, c, stream=None):
    _chk(_lib.pf_page_mtimes(_dt(a), C.byref(A), _p(a), int(transA), C.byref(B), _p(b), int(transB), C.byref(Cd),
                             _p(c), _s(stream)), "pf_page_mtimes")


def page_mv(A: Pages, a, transA, X: Pages, x, Y: Pages, y, stream=None):
    _chk(_lib.pf_page_mv(_dt(a), C.byref(A), _p(a), int(transA), C.byref(X), _p(x), C.byref(Y), _p(y), _s(stream)),
         "pf_page_mv")


def page_scale(s, s_stride, A: Pages, a, Cd: Pages, c, stream=None):
    _chk(_lib.pf_page_scale(_dt(a), _p(s), int(s_stride), C.byref(A), _p(a), C.byref(Cd), _p(c), _s(stream)),
         "pf_page_scale")


def page_bilinear(U: Pages, u, A: Pages, a, V: Pages, v, q, stream=None):
    _chk(_lib.pf_page_bilinear(_dt(a), C.byref(U), _p(u), C.byref(A), _p(a), C.byref(V), _p(v), _p(q), _s(stream)),
         "pf_page_bilinear")


# ----------------------------------------------------------------------------- elements
def _mesh(coords, elems):
    if coords.dtype != torch.float64 or elems.dtype != torch.int32:
        raise ValueError("coords must be float64 and elems int32")
    if not (coords.is_contiguous() and elems.is_contiguous()):
        raise ValueError("coords and elems must be contiguous")
    return coords.shape[0], coords.shape[1], elems.shape[0]


def elem_geometry(prec, coords, elems, det=None, vol=None, grads=None, normals=None, facet=None, fb=None,
                  flags=None, counters=None, stream=None):
    nn, dim, ne = _mesh(coords, elems)
    _chk(_lib.pf_elem_geometry(dim, prec, nn, _p(coords), ne, _p(elems), _p(det), _p(vol), _p(grads), _p(normals),
                               _p(facet), _ref(fb, Fallback), _p(flags), _p(counters), _s(stream)),
         "pf_elem_geometry")


def elem_stiffness_mass(prec, coords, elems, cK=None, cM=None, K3D=None, M3D=None, fb=None, flags=None,
                        counters=None, stream=None):
    nn, dim, ne = _mesh(coords, elems)
    _chk(_lib.pf_elem_stiffness_mass(dim, prec, nn, _p(coords), ne, _p(elems), _p(cK), _p(cM), _p(K3D), _p(M3D),
                                     _ref(fb, Fallback), _p(flags), _p(counters), _s(stream)),
         "pf_elem_stiffness_mass")


def boundary_normals(prec, coords, faces, unit=None, measure=None, stream=None):
    nn, dim = coords.shape
    if coords.dtype != torch.float64 or faces.dtype != torch.int32:
        raise ValueError("coords must be float64 and faces int32")
    _chk(_lib.pf_boundary_normals(dim, prec, nn, _p(coords), faces.shape[0], _p(faces), _p(unit), _p(measure),
                                  _s(stream)), "pf_boundary_normals")


def quad_count(dim, order):
    if dim not in (2, 3) or order not in (1, 2):
        raise ValueError("dim must be 2 or 3 and order 1 or 2")
    return 1 if order == 1 else dim + 1


def quad_points(coords, elems, order, xq=None, stream=None):
    """Integration points (ne, nq, dim) FP64 of the order-1 / order-2 rule of every element."""
    nn, dim = coords.shape
    ne = elems.shape[0]
    if xq is None:
        xq = torch.empty((ne, quad_count(dim, order), dim), dtype=torch.float64, device=coords.device)
    _chk(_lib.pf_quad_points(dim, int(order), nn, _p(coords), ne, _p(elems), _p(xq), _s(stream)), "pf_quad_points")
    return xq


# ----------------------------------------------------------------------------- assembly
class Csr:
    """Owner of a pf_csr handle (CSR structure of one P1 mesh)."""

    def __init__(self):
        h = P()
        _chk(_lib.pf_csr_create(C.byref(h)), "pf_csr_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def symbolic(self, dim, nn, elems, stream=None):
        if elems.dtype != torch.int32 or not elems.is_contiguous():
            raise ValueError("elems must be contiguous int32")
        self._dim = int(dim)
        _chk(_lib.pf_csr_symbolic(self._h, int(dim), int(nn), elems.shape[0], _p(elems), _s(stream)),
             "pf_csr_symbolic")
        return self

    def symbolic_p2(self, dim, nn, elems2, stream=None):
        """Structure of a P2 mesh (elems2: ne x 6 or 10 int32)."""
        if elems2.dtype != torch.int32 or not elems2.is_contiguous():
            raise ValueError("elems2 must be contiguous int32")
        self._dim = int(dim)
        _chk(_lib.pf_csr_symbolic_p2(self._h, int(dim), int(nn), elems2.shape[0], _p(elems2), _s(stream)),
             "pf_csr_symbolic_p2")
        return self

    def assemble_pages(self, prec, pagesK=None, pagesM=None, valsK=None, valsM=None, stream=None):
        """sparse() of element pages (ne x nlb x nlb column-major) into valsK / valsM (nnz)."""
        _chk(_lib.pf_csr_assemble_pages(self._h, prec, _p(pagesK), _p(pagesM), _p(valsK), _p(valsM), _s(stream)),
             "pf_csr_assemble_pages")

    def info(self):
        nn, nnz, rp, ci = I64(), I64(), P(), P()
        _chk(_lib.pf_csr_info(self._h, C.byref(nn), C.byref(nnz), C.byref(rp), C.byref(ci)), "pf_csr_info")
        return nn.value, nnz.value, rp.value, ci.value

    def memory(self):
        """(resident device bytes of the structure, build scratch still held)"""
        res, scr = I64(), I64()
        _chk(_lib.pf_csr_memory(self._h, C.byref(res), C.byref(scr)), "pf_csr_memory")
        return res.value, scr.value

    def numeric_info(self, prec):
        """(rows per workgroup of the numeric launch, largest number of elements around a node)"""
        rows, madj = I32(), I32()
        _chk(_lib.pf_csr_numeric_info(self._h, prec, C.byref(rows), C.byref(madj)), "pf_csr_numeric_info")
        return rows.value, madj.value

    CSR_STAGES = ("adjacency", "pattern", "row offsets", "columns")

    def set_timing(self, on=True):
        """Record per-stage events in every later symbolic call (and clear the sums)."""
        _chk(_lib.pf_csr_set_timing(self._h, 1 if on else 0), "pf_csr_set_timing")

    def stage_times(self):
        """({stage: summed ms}, calls) since timing was switched on."""
        ms = (C.c_double * len(self.CSR_STAGES))()
        calls = I64()
        _chk(_lib.pf_csr_stage_times(self._h, ms, C.byref(calls)), "pf_csr_stage_times")
        return dict(zip(self.CSR_STAGES, list(ms))), calls.value

    def structure(self, stream=None):
        """Copies of (row_ptr, col_idx) as int32 device tensors."""
        nn, nnz, rp, ci = self.info()
        row_ptr = torch.empty(nn + 1, dtype=torch.int32, device="cuda")
        col_idx = torch.empty(max(nnz, 1), dtype=torch.int32, device="cuda")[:nnz]
        _memcpy_d2d(row_ptr.data_ptr(), rp, 4 * (nn + 1), stream)
        if nnz:
            _memcpy_d2d(col_idx.data_ptr(), ci, 4 * nnz, stream)
        return row_ptr, col_idx

    def assemble(self, prec, coords, elems, valsK, valsM=None, cK=None, cM=None, fb=None, counters=None,
                 stream=None):
        _chk(_lib.pf_assemble(self._h, prec, _p(coords), _p(elems), _p(cK), _p(cM), _p(valsK), _p(valsM),
                              _ref(fb, Fallback), _p(counters), _s(stream)), "pf_assemble")

    def assemble_quad(self, prec, coords, order, valsK, valsM=None, cKq=None, cMq=None, fb=None, counters=None,
                      stream=None):
        """Assembly with coefficients at the integration points (ne x nq, type prec)."""
        _chk(_lib.pf_assemble_quad(self._h, prec, _p(coords), int(order), _p(cKq), _p(cMq), _p(valsK), _p(valsM),
                                   _ref(fb, Fallback), _p(counters), _s(stream)), "pf_assemble_quad")

    def faces(self, coords, elems, stream=None):
        """Build the face lists (all faces, boundary faces) of the structure's mesh."""
        _chk(_lib.pf_csr_faces(self._h, _p(coords), _p(elems), _s(stream)), "pf_csr_faces")
        return self

    def face_lists(self, stream=None):
        """Copies of (faces, fel, bfaces, bel) as int32 device tensors."""
        nf, nfb = I64(), I64()
        f, fe, bf, be = P(), P(), P(), P()
        _chk(_lib.pf_csr_faces_info(self._h, C.byref(nf), C.byref(nfb), C.byref(f), C.byref(fe), C.byref(bf),
                                    C.byref(be)), "pf_csr_faces_info")
        dim = self._dim
        out = []
        for ptr, n in ((f, nf.value * dim), (fe, 2 * nf.value), (bf, nfb.value * dim), (be, nfb.value)):
            t = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")[:n]
            if n:
                _memcpy_d2d(t.data_ptr(), ptr.value, 4 * n, stream)
            out.append(t)
        return (out[0].view(-1, dim), out[1].view(-1, 2), out[2].view(-1, dim), out[3])

    def rhs(self, prec, coords, elems, order, fq, b2D, b=None, fb=None, counters=None, stream=None):
        """Load vector: local vectors into b2D (ne x nlb) and, if b is given, their node sums."""
        _chk(_lib.pf_rhs(self._h, prec, _p(coords), _p(elems), int(order), _p(fq), _p(b2D), _p(b),
                         _ref(fb, Fallback), _p(counters), _s(stream)), "pf_rhs")

    def energies(self, prec, coords, elems, order, u, cKq=None, cMq=None, b2D=None, J=None, totals=None, fb=None,
                 counters=None, stream=None):
        """Local energy parts into J (3 x ne) and/or their FP64 sums into totals (3 doubles)."""
        _chk(_lib.pf_energies(self._h, prec, _p(coords), _p(elems), int(order), _p(cKq), _p(cMq), _p(u), _p(b2D),
                              _p(J), _p(totals), _ref(fb, Fallback), _p(counters), _s(stream)), "pf_energies")

    def energies_noalloc(self, prec, coords, elems, order, u, cKq=None, cMq=None, b2D=None, J=None, totals=None,
                         fb=None, counters=None, stream=None):
        """energies() with the block sums in the library's static per-device array (no allocation)."""
        _chk(_lib.pf_energies_noalloc(self._h, prec, _p(coords), _p(elems), int(order), _p(cKq), _p(cMq), _p(u),
                                      _p(b2D), _p(J), _p(totals), _ref(fb, Fallback), _p(counters), _s(stream)),
             "pf_energies_noalloc")

    def close(self):
        if self._h:
            _lib.pf_csr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


RULE_MAX = 64
GI_WORK = 2048


def simplex_points(coords, cells, lam, stream=None):
    """Points of the rule with barycentric points lam (nq x nv) on every cell: (nc, nq, dim) FP64."""
    import numpy as np
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    nc, nv = cells.shape
    nq = lam.shape[0]
    dim = coords.shape[1]
    X = torch.empty((nc, nq, dim), dtype=torch.float64, device="cuda")
    _chk(_lib.pf_simplex_points(dim, nv, coords.shape[0], _p(coords), nc, _p(cells), nq,
                                lam.ctypes.data_as(P), _p(X), _s(stream)), "pf_simplex_points")
    return X


P2_RULE_MAX = 32


def p2_elements(prec, coords, elems2, ruleK=None, ruleM=None, cKq=None, cMq=None, K3D=None, M3D=None, fb=None,
                counters=None, stream=None):
    """P2 element matrices into K3D / M3D (ne x nlb2^2 pages); rules are (lam, w) host arrays."""
    import numpy as np

    def rule(r):
        if r is None:
            return 0, None, None, None
        lam = np.ascontiguousarray(r[0], dtype=np.float64)
        w = np.ascontiguousarray(r[1], dtype=np.float64)
        return lam.shape[0], lam, w, (lam, w)
    nqK, lK, wK, keepK = rule(ruleK)
    nqM, lM, wM, keepM = rule(ruleM)
    nn, dim = coords.shape
    _chk(_lib.pf_p2_elements(dim, prec, nn, _p(coords), elems2.shape[0], _p(elems2), nqK,
                             None if lK is None else lK.ctypes.data_as(P), None if wK is None else wK.ctypes.data_as(P),
                             _p(cKq), nqM, None if lM is None else lM.ctypes.data_as(P),
                             None if wM is None else wM.ctypes.data_as(P), _p(cMq), _p(K3D), _p(M3D),
                             _ref(fb, Fallback), _p(counters), _s(stream)), "pf_p2_elements")


def gi(prec, fip, w, sizes, normals=None, value=None, work=None, stream=None):
    """The GI function; returns the device FP64 scalar tensor `value`."""
    import numpy as np
    w = np.ascontiguousarray(w, dtype=np.float64)
    nc, nq = fip.shape[0], fip.shape[1]
    d = fip.shape[2] if fip.dim() == 3 else 1
    value = value if value is not None else torch.empty(1, dtype=torch.float64, device="cuda")
    work = work if work is not None else torch.empty(GI_WORK, dtype=torch.float64, device="cuda")
    _chk(_lib.pf_gi(prec, nc, nq, d, _p(fip), w.ctypes.data_as(P), _p(sizes), _p(normals), _p(value), _p(work),
                    _s(stream)), "pf_gi")
    return value


# ----------------------------------------------------------------------- batch plans
class Plan:
    """Owner of a pf_plan handle: inverse and product of many groups of pages in one
    persistent launch replayed from a HIP graph.  `groups` are dicts with keys order, ops,
    a, b, x, c, det (tensors, b/x/c/det optional) or pf_group structures."""

    def __init__(self, dtype, max_groups, fb=None):
        h = P()
        _chk(_lib.pf_plan_create(dtype, int(max_groups), _ref(fb, Fallback), C.byref(h)), "pf_plan_create")
        self._h = h
        self._keep = None

    def set_groups(self, groups):
        arr = (Group * max(len(groups), 1))()
        keep = []
        for i, g in enumerate(groups):
            if isinstance(g, Group):
                arr[i] = g
                continue
            a = g["a"]
            keep.append(g)
            arr[i] = Group(int(g["order"]), int(g["ops"]), int(g.get("count", a.numel() // g["order"] ** 2)),
                           _p(a), _p(g.get("b")), _p(g.get("x")), _p(g.get("c")), _p(g.get("det")))
        _chk(_lib.pf_plan_set_groups(self._h, arr, len(groups)), "pf_plan_set_groups")
        self._keep = keep  # the tensors stay alive while the plan may run on them
        return self

    def schedule(self):
        s = Schedule()
        _chk(_lib.pf_plan_get_schedule(self._h, C.byref(s)), "pf_plan_get_schedule")
        return s

    def set_schedule(self, waves, per_order):
        """per_order: {order: (lanes, staged, tile)}; orders not given keep (1, 1, 1)."""
        s = Schedule()
        s.waves = int(waves)
        for n in range(5):
            s.order[n] = OrderSchedule(*per_order.get(n, (1, 1, 1)))
        _chk(_lib.pf_plan_set_schedule(self._h, C.byref(s)), "pf_plan_set_schedule")

    def tune(self, cache_path=None, mode=TUNE_CACHED, stream=None):
        path = None if cache_path is None else os.fsencode(cache_path)
        _chk(_lib.pf_plan_tune(self._h, path, int(mode), _s(stream)), "pf_plan_tune")
        return self.schedule()

    def run(self, counters=None, stream=None):
        _chk(_lib.pf_plan_run(self._h, _p(counters), _s(stream)), "pf_plan_run")

    def launch(self, counters=None, stream=None):
        _chk(_lib.pf_plan_launch(self._h, _p(counters), _s(stream)), "pf_plan_launch")

    def info(self):
        nt, grid, lds = I64(), I32(), I32()
        _chk(_lib.pf_plan_info(self._h, C.byref(nt), C.byref(grid), C.byref(lds)), "pf_plan_info")
        return nt.value, grid.value, lds.value

    def close(self):
        if self._h:
            _lib.pf_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------- serving
def _host_ptr(x):
    """Address of a host array: a CPU torch tensor (pinned for asynchronous copies) or a
    C-contiguous numpy array."""
    if x is None:
        return None
    if isinstance(x, torch.Tensor):
        if x.is_cuda or not x.is_contiguous():
            raise ValueError("server job arrays must be contiguous host tensors")
        return x.data_ptr()
    if not x.flags["C_CONTIGUOUS"]:
        raise ValueError("server job arrays must be C-contiguous")
    return x.ctypes.data


def server_footprint(dim, prec, nn, ne):
    """Device bytes a job of this size is admitted with when its structure is not resident."""
    job = Job(int(dim), int(prec), int(nn), int(ne), 16, 16, 0, -1.0, fallback(), None, None, 0)
    b = C.c_size_t()
    _chk(_lib.pf_server_footprint(C.byref(job), C.byref(b)), "pf_server_footprint")
    return b.value


class Server:
    """Owner of a pf_server handle: assembly and page-op jobs from host memory, admitted by a
    device memory budget, batched per scheduler tick, with resident structures per topology."""

    def __init__(self, hbm_budget, max_slots=256, flags=0):
        h = P()
        _chk(_lib.pf_server_create(int(hbm_budget), int(max_slots), int(flags), C.byref(h)), "pf_server_create")
        self._h = h
        self._keep = {}

    def now(self):
        return _lib.pf_server_now(self._h)

    def submit(self, dim, prec, coords, elems, topology=0, arrival=-1.0, fb=None, valsK=None, valsM=None):
        nn, ne = coords.shape[0], elems.shape[0]
        cap = 0
        for v in (valsK, valsM):
            if v is not None:
                cap = v.shape[0] if cap == 0 else min(cap, v.shape[0])
        job = Job(int(dim), int(prec), nn, ne, _host_ptr(coords), _host_ptr(elems), int(topology), float(arrival),
                  fb if fb is not None else fallback(), _host_ptr(valsK), _host_ptr(valsM), cap)
        t = C.c_uint64()
        _chk(_lib.pf_server_submit(self._h, C.byref(job), C.byref(t)), "pf_server_submit")
        self._keep[t.value] = (coords, elems, valsK, valsM)  # alive until the job is done
        return t.value

    def submit_pages(self, prec, order, ops, a, b=None, x=None, c=None, det=None, arrival=-1.0):
        """A page-op job: count n x n pages a (and b) in host memory (paper layout); outputs
        inv(a) into x, a*b into c, det(a) into det (host arrays, each nullable)."""
        count = a.shape[0]
        job = Job()
        job.kind = JOB_PAGES
        job.prec = int(prec)
        job.order = int(order)
        job.ops = int(ops)
        job.count = int(count)
        job.arrival = float(arrival)
        job.a, job.b, job.x, job.c, job.det = (_host_ptr(v) for v in (a, b, x, c, det))
        t = C.c_uint64()
        _chk(_lib.pf_server_submit(self._h, C.byref(job), C.byref(t)), "pf_server_submit")
        self._keep[t.value] = (a, b, x, c, det)
        return t.value

    def poll(self, ticket):
        r = JobResult()
        _chk(_lib.pf_server_poll(self._h, ticket, C.byref(r)), "pf_server_poll")
        if r.done:
            self._keep.pop(ticket, None)
        return r.as_dict()

    def wait(self, ticket):
        r = JobResult()
        _chk(_lib.pf_server_wait(self._h, ticket, C.byref(r)), "pf_server_wait")
        self._keep.pop(ticket, None)
        return r.as_dict()

    def drain(self):
        _chk(_lib.pf_server_drain(self._h), "pf_server_drain")
        self._keep.clear()

    def stats(self):
        s = Stats()
        _chk(_lib.pf_server_stats(self._h, C.byref(s)), "pf_server_stats")
        return s.as_dict()

    def close(self):
        if self._h:
            _lib.pf_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_hip = None


def _memcpy_d2d(dst, src, nbytes, stream=None):
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpyAsync.argtypes = [P, P, C.c_size_t, C.c_int, P]
        _hip.hipMemcpyAsync.restype = C.c_int
    rc = _hip.hipMemcpyAsync(P(dst), P(src), nbytes, 3, _s(stream))  # hipMemcpyDeviceToDevice
    if rc != 0:
        raise RuntimeError(f"hipMemcpyAsync failed ({rc})")
