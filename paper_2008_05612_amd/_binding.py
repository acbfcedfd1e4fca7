"""ctypes marshalling for libhpmap.so; names mirror the C entry points of hp.h.

Device buffers are torch tensors on the GPU; their ``data_ptr()`` is passed
through unchanged.  ``stream`` arguments accept a ``torch.cuda.Stream`` (or
None for torch's current stream).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libhpmap.so")

FORM_POPCOUNT = 0
FORM_GEMM_I8 = 1
FORM_BLOCKED_I8 = 2
NONE = 0xFFFF

_STATUS = {0: "HP_OK", -1: "HP_EINVAL", -2: "HP_ENOMEM", -3: "HP_EDEVICE", -4: "HP_ERANGE",
           -5: "HP_EUNSUPPORTED"}


class LibraryMissing(RuntimeError):
    pass


class HPError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        self.status = status
        super().__init__("%s failed with %s: %s" % (where, _STATUS.get(status, status), msg))


class _Info(ctypes.Structure):
    _fields_ = [("X", ctypes.c_int32), ("Y", ctypes.c_int32), ("Z", ctypes.c_int32),
                ("N", ctypes.c_int32), ("group_order", ctypes.c_uint32),
                ("n_walks", ctypes.c_uint64), ("n_conf", ctypes.c_uint32),
                ("n_class", ctypes.c_uint32), ("n_selfrev", ctypes.c_uint32),
                ("nbp", ctypes.c_uint32), ("K", ctypes.c_uint32), ("W", ctypes.c_uint32),
                ("K_pad", ctypes.c_uint32), ("table", ctypes.c_int32 * 4),
                ("unary_rows", ctypes.c_uint32), ("cmax", ctypes.c_uint32)]


class _Job(ctypes.Structure):
    _fields_ = [("structs", ctypes.c_void_p), ("d_ws", ctypes.c_void_p),
                ("seq_lo", ctypes.c_uint64), ("seq_hi", ctypes.c_uint64),
                ("d_out", ctypes.c_void_p), ("d_emin", ctypes.c_void_p),
                ("d_designability", ctypes.c_void_p), ("d_nondesign", ctypes.c_void_p)]


_lib = None


def library_path() -> str:
    return _LIB_PATH


def library():
    """The loaded libhpmap.so; raises LibraryMissing if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise LibraryMissing("libhpmap.so is not built (python -m paper_2008_05612_amd.build)")
    L = ctypes.CDLL(_LIB_PATH)
    vp, i32, u64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_size_t
    st = ctypes.c_int
    sigs = {
        "hp_structures": (st, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(vp)]),
        "hp_structures_energy": (st, [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(vp)]),
        "hp_structs_free": (None, [vp]),
        "hp_structs_info": (st, [vp, ctypes.POINTER(_Info)]),
        "hp_structs_export": (st, [vp, vp, vp, vp, vp, vp, vp]),
        "hp_workspace_bytes": (sz, [vp]),
        "hp_upload": (st, [vp, vp, sz, vp]),
        "hp_enumerate": (st, [vp, vp, ctypes.c_int, u64, u64, vp, vp, vp, vp, vp]),
        "hp_batch_workspace_bytes": (sz, [ctypes.c_int]),
        "hp_canonical_count": (u64, [vp]),
        "hp_enumerate_symmetric": (st, [vp, vp, ctypes.c_int, u64, u64, vp, vp, vp, vp, vp]),
        "hp_canonical_block_count": (u64, [vp]),
        "hp_enumerate_symmetric_blocked": (st, [vp, vp, u64, u64, vp, vp, vp, vp, vp]),
        "hp_wide_block_count": (u64, [vp]),
        "hp_enumerate_symmetric_wide": (st, [vp, vp, u64, u64, vp, vp, vp, vp, vp]),
        "hp_enumerate_gap": (st, [vp, vp, ctypes.c_int, u64, u64, i32, vp, vp, vp, vp, vp, vp]),
        "hp_sample": (st, [vp, vp, ctypes.c_int, u64, u64, u64, i32, vp, vp, vp, vp, vp, vp, vp]),
        "hp_enumerate_batch": (st, [ctypes.POINTER(_Job), ctypes.c_int, ctypes.c_int, vp, sz, vp]),
        "hp_graph_capture_batch": (st, [ctypes.POINTER(_Job), ctypes.c_int, ctypes.c_int, vp, sz,
                                        ctypes.POINTER(vp)]),
        "hp_enumerate_batch_static": (st, [ctypes.POINTER(_Job), ctypes.c_int, ctypes.c_int, vp]),
        "hp_graph_launch": (st, [vp, vp]),
        "hp_graph_free": (None, [vp]),
        "hp_neighbors": (st, [vp, vp, vp, vp, vp, i32, vp, vp]),
        "hp_phi_counts": (st, [vp, vp, vp, vp]),
        "hp_phi_sparse": (st, [vp, vp, vp, vp, vp, u64, ctypes.POINTER(u64), vp]),
        "hp_components": (st, [vp, vp, vp, vp, vp, vp, vp]),
        "hp_blocked_select": (st, [ctypes.c_int, ctypes.c_int]),
        "hp_autotune_blocked": (st, [vp, vp, u64, u64, ctypes.c_int, ctypes.POINTER(ctypes.c_float),
                                     ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                     vp]),
        "hp_blocked_selected": (None, [ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
        "hp_gemm_shape_count": (ctypes.c_int, [ctypes.c_uint32]),
        "hp_gemm_shape_info": (st, [ctypes.c_uint32, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                    ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
        "hp_gemm_select": (st, [ctypes.c_uint32, ctypes.c_int]),
        "hp_gemm_selected": (ctypes.c_int, [ctypes.c_uint32]),
        "hp_autotune": (st, [vp, vp, u64, u64, ctypes.c_int, ctypes.POINTER(ctypes.c_float),
                             ctypes.POINTER(ctypes.c_int), vp]),
        "hp_last_error": (ctypes.c_char_p, []),
        "hp_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sigs.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(status: int, where: str):
    if status != 0:
        msg = library().hp_last_error().decode()
        raise HPError(status, where, msg)


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _u16_dtypes():
    import torch
    return (torch.int16, torch.uint16) if hasattr(torch, "uint16") else (torch.int16,)


_U16 = object()   # marker: int16 or uint16 tensors hold 16-bit phenotype ids


def _ptr(t, dtype=None, numel: Optional[int] = None, name: str = "buffer"):
    """Device pointer of an optional torch tensor, with dtype/size checks."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if dtype is _U16:
        dtype = _u16_dtypes()
    if dtype is not None:
        ok = t.dtype in dtype if isinstance(dtype, tuple) else t.dtype == dtype
        if not ok:
            raise ValueError("%s must have dtype %s, got %s" % (name, dtype, t.dtype))
    if numel is not None and t.numel() < numel:
        raise ValueError("%s needs >= %d elements, has %d" % (name, numel, t.numel()))
    return t.data_ptr()


class Structures:
    """Owning wrapper of an hp_structs handle (host-side tables)."""

    def __init__(self, X: int, Y: int, Z: int = 1, table=None):
        h = ctypes.c_void_p()
        if table is None:
            _check(library().hp_structures(X, Y, Z, ctypes.byref(h)), "hp_structures")
        else:
            t = (ctypes.c_int32 * 4)(*[int(x) for x in table])
            _check(library().hp_structures_energy(X, Y, Z, t, ctypes.byref(h)),
                   "hp_structures_energy")
        self._h = h
        info = _Info()
        _check(library().hp_structs_info(h, ctypes.byref(info)), "hp_structs_info")
        for name, _ in _Info._fields_:
            v = getattr(info, name)
            setattr(self, name, tuple(v) if name == "table" else int(v))
        self.dims = (X, Y, Z)
        self._ws = None

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.hp_structs_free(h)
            self._h = None

    def export(self) -> dict:
        N, nc, nq, K, nbp = self.N, self.n_conf, self.n_class, self.K, self.nbp
        walks = np.zeros((nc, N), np.uint8)
        c2q = np.zeros(nc, np.uint16)
        rev = np.zeros(nc, np.uint32)
        srev = np.zeros(max(nq, 1), np.uint8)
        pairs = np.zeros((max(K, 1), 2), np.uint8)
        contacts = np.zeros((nc, max(nbp, 1), 2), np.uint8)
        _check(library().hp_structs_export(self._h, walks.ctypes.data, c2q.ctypes.data,
                                           rev.ctypes.data, srev.ctypes.data, pairs.ctypes.data,
                                           contacts.ctypes.data), "hp_structs_export")
        return {"walks": walks, "conf_to_class": c2q, "rev_conf": rev, "self_rev": srev[:nq],
                "pairs": pairs[:K], "contacts": contacts[:, :nbp]}

    def workspace(self, device="cuda", stream=None):
        """Device workspace (uint8 tensor) with this handle's tables uploaded."""
        import torch
        if self._ws is None:
            nbytes = hp_workspace_bytes(self)
            ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
            off = (-ws.data_ptr()) % 256
            ws = ws[off:off + nbytes]
            hp_upload(self, ws, stream)
            torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
            self._ws = ws
        return self._ws


def hp_structures(X: int, Y: int, Z: int = 1, table=None) -> Structures:
    """Structures of the X*Y*Z box; `table` = {E_PP, E_PH, E_HP, E_HH} or None
    for pure HP (hp_structures_energy / hp_structures)."""
    return Structures(X, Y, Z, table)


def hp_workspace_bytes(s: Structures) -> int:
    return int(library().hp_workspace_bytes(s.handle))


def hp_upload(s: Structures, ws, stream=None):
    import torch
    p = _ptr(ws, torch.uint8, hp_workspace_bytes(s), "workspace")
    _check(library().hp_upload(s.handle, p, ws.numel(), _stream_handle(stream)), "hp_upload")


def hp_enumerate(s: Structures, ws, form: int, seq_lo: int, seq_hi: int, out=None, emin=None,
                 designability=None, nondesign=None, stream=None):
    import torch
    n = seq_hi - seq_lo
    _check(library().hp_enumerate(
        s.handle, _ptr(ws, torch.uint8, None, "workspace"), form, seq_lo, seq_hi,
        _ptr(out, _U16, n, "out"),
        _ptr(emin, torch.int32, n, "emin"),
        _ptr(designability, torch.int64, s.n_class, "designability"),
        _ptr(nondesign, torch.int64, 1, "nondesign"),
        _stream_handle(stream)), "hp_enumerate")


def hp_autotune_blocked(s: Structures, ws, seq_lo: int = 0, n_seq: int = 1 << 20,
                        repeats: int = 2, stream=None):
    """Time the blocked-form launch shapes (9, plus wide blocks where they
    apply), select the fastest; returns ((nw, mode), [ms per shape in hp.h
    order; -1 for a shape that does not apply])."""
    import torch
    ms = (ctypes.c_float * 10)()
    nw, mode = ctypes.c_int(), ctypes.c_int()
    _check(library().hp_autotune_blocked(s.handle, _ptr(ws, torch.uint8, None, "workspace"), seq_lo,
                                         n_seq, repeats, ms, ctypes.byref(nw), ctypes.byref(mode),
                                         _stream_handle(stream)), "hp_autotune_blocked")
    return (nw.value, mode.value), list(ms)


def hp_canonical_block_count(s: Structures) -> int:
    return int(library().hp_canonical_block_count(s.handle))


def hp_enumerate_symmetric_blocked(s: Structures, ws, b_lo: int, b_hi: int, out=None, emin=None,
                                   designability=None, nondesign=None, stream=None):
    """Canonical blocks [b_lo, b_hi) of the blocked form; out / emin are full
    2^N maps indexed by sequence (written at s and, off the diagonal, at
    reverse(s))."""
    import torch
    n = 1 << s.N
    _check(library().hp_enumerate_symmetric_blocked(
        s.handle, _ptr(ws, torch.uint8, None, "workspace"), b_lo, b_hi,
        _ptr(out, _U16, n, "out"), _ptr(emin, torch.int32, n, "emin"),
        _ptr(designability, torch.int64, s.n_class, "designability"),
        _ptr(nondesign, torch.int64, 1, "nondesign"), _stream_handle(stream)),
        "hp_enumerate_symmetric_blocked")


def hp_wide_block_count(s: Structures) -> int:
    return int(library().hp_wide_block_count(s.handle))


def hp_enumerate_symmetric_wide(s: Structures, ws, b_lo: int, b_hi: int, out=None, emin=None,
                                designability=None, nondesign=None, stream=None):
    """Canonical wide blocks [b_lo, b_hi) (1024 sequences each); out / emin
    are full 2^N maps indexed by sequence (written at s and, off the
    diagonal, at reverse(s))."""
    import torch
    n = 1 << s.N
    _check(library().hp_enumerate_symmetric_wide(
        s.handle, _ptr(ws, torch.uint8, None, "workspace"), b_lo, b_hi,
        _ptr(out, _U16, n, "out"), _ptr(emin, torch.int32, n, "emin"),
        _ptr(designability, torch.int64, s.n_class, "designability"),
        _ptr(nondesign, torch.int64, 1, "nondesign"), _stream_handle(stream)),
        "hp_enumerate_symmetric_wide")


def hp_enumerate_gap(s: Structures, ws, form: int, seq_lo: int, seq_hi: int, threshold: int = 1,
                     out=None, emin=None, gap=None, designability=None, nondesign=None,
                     stream=None):
    """hp_enumerate with an energy-gap threshold and an optional uint8 gap map."""
    import torch
    n = seq_hi - seq_lo
    _check(library().hp_enumerate_gap(
        s.handle, _ptr(ws, torch.uint8, None, "workspace"), form, seq_lo, seq_hi, threshold,
        _ptr(out, _U16, n, "out"), _ptr(emin, torch.int32, n, "emin"),
        _ptr(gap, torch.uint8, n, "gap"),
        _ptr(designability, torch.int64, s.n_class, "designability"),
        _ptr(nondesign, torch.int64, 1, "nondesign"), _stream_handle(stream)), "hp_enumerate_gap")


def hp_sample(s: Structures, ws, form: int, seed: int, idx_lo: int, idx_hi: int,
              threshold: int = 1, seqs=None, out=None, emin=None, gap=None, designability=None,
              nondesign=None, stream=None):
    """Random-sampling mode: draws idx_lo .. idx_hi-1 of the device generator
    seeded with `seed`; per-draw outputs are indexed by draw - idx_lo."""
    import torch
    n = idx_hi - idx_lo
    _check(library().hp_sample(
        s.handle, _ptr(ws, torch.uint8, None, "workspace"), form, seed & (2**64 - 1), idx_lo,
        idx_hi, threshold, _ptr(seqs, torch.int64, n, "seqs"), _ptr(out, _U16, n, "out"),
        _ptr(emin, torch.int32, n, "emin"), _ptr(gap, torch.uint8, n, "gap"),
        _ptr(designability, torch.int64, s.n_class, "designability"),
        _ptr(nondesign, torch.int64, 1, "nondesign"), _stream_handle(stream)), "hp_sample")


def hp_blocked_select(nw: int, mode: int = -1):
    """Launch shape of the blocked int8 form: waves per workgroup (2, 4 or 8)
    and staging mode (0 double-buffered, 1 pipelined, 2 operand in LDS, 3 wide
    blocks of 1024 sequences (nw 4), -1 by product depth)."""
    _check(library().hp_blocked_select(nw, mode), "hp_blocked_select")


def hp_blocked_selected():
    """(nw, mode) of the blocked int8 form."""
    nw, mode = ctypes.c_int(), ctypes.c_int()
    library().hp_blocked_selected(ctypes.byref(nw), ctypes.byref(mode))
    return nw.value, mode.value


def hp_canonical_count(s: Structures) -> int:
    return int(library().hp_canonical_count(s.handle))


def hp_enumerate_symmetric(s: Structures, ws, form: int, t_lo: int, t_hi: int, out=None,
                           emin=None, designability=None, nondesign=None, stream=None):
    """Canonical sequences with index in [t_lo, t_hi); out / emin are full
    2^N maps indexed by sequence (written at s and reverse(s))."""
    import torch
    n = 1 << s.N
    _check(library().hp_enumerate_symmetric(
        s.handle, _ptr(ws, torch.uint8, None, "workspace"), form, t_lo, t_hi,
        _ptr(out, _U16, n, "out"), _ptr(emin, torch.int32, n, "emin"),
        _ptr(designability, torch.int64, s.n_class, "designability"),
        _ptr(nondesign, torch.int64, 1, "nondesign"), _stream_handle(stream)),
        "hp_enumerate_symmetric")


@dataclass
class Job:
    structs: Structures
    ws: object
    seq_lo: int
    seq_hi: int
    out: object = None
    emin: object = None
    designability: object = None
    nondesign: object = None


def _jobs_array(jobs: Sequence[Job]):
    import torch
    arr = (_Job * len(jobs))()
    for i, j in enumerate(jobs):
        n = j.seq_hi - j.seq_lo
        arr[i] = _Job(j.structs.handle.value, _ptr(j.ws, torch.uint8, None, "workspace"), j.seq_lo,
                      j.seq_hi, _ptr(j.out, _U16, n, "out"), _ptr(j.emin, torch.int32, n, "emin"),
                      _ptr(j.designability, torch.int64, j.structs.n_class, "designability"),
                      _ptr(j.nondesign, torch.int64, 1, "nondesign"))
    return arr


def batch_workspace_bytes(njobs: int) -> int:
    return int(library().hp_batch_workspace_bytes(njobs))


def hp_enumerate_batch(jobs: Sequence[Job], form: int, batch_ws, stream=None):
    import torch
    arr = _jobs_array(jobs)
    _check(library().hp_enumerate_batch(arr, len(jobs), form,
                                        _ptr(batch_ws, torch.uint8,
                                             batch_workspace_bytes(len(jobs)), "batch workspace"),
                                        batch_ws.numel(), _stream_handle(stream)),
           "hp_enumerate_batch")


STATIC_BATCH_MAX_JOBS = 32   # HP_STATIC_BATCH_MAX_JOBS


def hp_enumerate_batch_static(jobs: Sequence[Job], form: int, stream=None):
    """hp_enumerate_batch without a workspace: the work list goes to the
    library's own device array (no allocation; at most 32 jobs)."""
    arr = _jobs_array(jobs)
    _check(library().hp_enumerate_batch_static(arr, len(jobs), form, _stream_handle(stream)),
           "hp_enumerate_batch_static")


class Graph:
    def __init__(self, handle, keep):
        self._h = handle
        self._keep = keep   # buffers referenced by the captured work list

    def launch(self, stream=None):
        _check(library().hp_graph_launch(self._h, _stream_handle(stream)), "hp_graph_launch")

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hp_graph_free(self._h)
            self._h = None


def hp_graph_capture_batch(jobs: Sequence[Job], form: int, batch_ws) -> Graph:
    import torch
    arr = _jobs_array(jobs)
    h = ctypes.c_void_p()
    _check(library().hp_graph_capture_batch(arr, len(jobs), form,
                                            _ptr(batch_ws, torch.uint8,
                                                 batch_workspace_bytes(len(jobs)),
                                                 "batch workspace"),
                                            batch_ws.numel(), ctypes.byref(h)),
           "hp_graph_capture_batch")
    return Graph(h, (list(jobs), batch_ws))


def hp_neighbors(s: Structures, phen_map, neutral=None, deleterious=None, other=None,
                 phi_q: int = -1, phi_row=None, stream=None):
    import torch
    _check(library().hp_neighbors(
        s.handle, _ptr(phen_map, _U16, 1 << s.N, "map"),
        _ptr(neutral, torch.int64, s.n_class, "neutral"),
        _ptr(deleterious, torch.int64, s.n_class, "deleterious"),
        _ptr(other, torch.int64, s.n_class, "other"), phi_q,
        _ptr(phi_row, torch.int64, s.n_class + 1, "phi_row"), _stream_handle(stream)),
        "hp_neighbors")


def hp_phi_counts(s: Structures, phen_map, counts, stream=None):
    """Add the phi_pq numerators of every phenotype pair to `counts`, an int64
    device tensor of n_class x (n_class + 1) (last column: deleterious)."""
    import torch
    _check(library().hp_phi_counts(
        s.handle, _ptr(phen_map, _U16, 1 << s.N, "map"),
        _ptr(counts, torch.int64, s.n_class * (s.n_class + 1), "counts"),
        _stream_handle(stream)), "hp_phi_counts")


def hp_phi_sparse(s: Structures, counts, row_ptr, cols=None, vals=None, stream=None) -> int:
    """Compressed rows of a counts matrix; returns the number of non-zero
    entries.  cols (int32) / vals (int64) None: size query only."""
    import torch
    cap = 0 if cols is None else min(cols.numel(), vals.numel() if vals is not None else 0)
    nnz = ctypes.c_uint64(0)
    _check(library().hp_phi_sparse(
        s.handle, _ptr(counts, torch.int64, s.n_class * (s.n_class + 1), "counts"),
        _ptr(row_ptr, torch.int64, s.n_class + 1, "row_ptr"), _ptr(cols, torch.int32, None, "cols"),
        _ptr(vals, torch.int64, None, "vals"), cap, ctypes.byref(nnz), _stream_handle(stream)),
        "hp_phi_sparse")
    return int(nnz.value)


def hp_components(s: Structures, phen_map, labels, compsize, ncomp=None, largest=None,
                  stream=None):
    import torch
    n = 1 << s.N
    _check(library().hp_components(
        s.handle, _ptr(phen_map, _U16, n, "map"), _ptr(labels, torch.int32, n, "labels"),
        _ptr(compsize, torch.int32, n, "compsize"), _ptr(ncomp, torch.int32, s.n_class, "ncomp"),
        _ptr(largest, torch.int32, s.n_class, "largest"), _stream_handle(stream)),
        "hp_components")


def hp_gemm_shapes(K_pad: int):
    """Compiled tile shapes of the int8 form for one product depth, as
    (T, NW, mode) tuples in library order."""
    L = library()
    out = []
    for i in range(L.hp_gemm_shape_count(K_pad)):
        T, NW, mode = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(L.hp_gemm_shape_info(K_pad, i, ctypes.byref(T), ctypes.byref(NW),
                                    ctypes.byref(mode)), "hp_gemm_shape_info")
        out.append((T.value, NW.value, mode.value))
    return out


def hp_gemm_select(K_pad: int, idx: int):
    _check(library().hp_gemm_select(K_pad, idx), "hp_gemm_select")


def hp_gemm_selected(K_pad: int) -> int:
    return int(library().hp_gemm_selected(K_pad))


def hp_autotune(s: Structures, ws, seq_lo: int, n_seq: int, repeats: int = 2, stream=None):
    """Time every compiled shape of s.K_pad on [seq_lo, seq_lo+n_seq), select the
    fastest; returns (best index, list of milliseconds per shape)."""
    import torch
    n = library().hp_gemm_shape_count(s.K_pad)
    ms = (ctypes.c_float * max(n, 1))()
    best = ctypes.c_int(-1)
    _check(library().hp_autotune(s.handle, _ptr(ws, torch.uint8, None, "workspace"), seq_lo,
                                 n_seq, repeats, ms, ctypes.byref(best), _stream_handle(stream)),
           "hp_autotune")
    return best.value, [float(ms[i]) for i in range(n)]
