"""ctypes binding of libcrp (include/crp.h): argument marshalling only.

Every step of the propagation runs in the library's HIP kernels; this module
only allocates device memory through PyTorch, fills the C descriptors and
calls the entry points of the same names on the current torch stream.  If the
library is missing or fails to load, every call raises: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcrp.so")

CRP_OK, CRP_ERR_INVALID, CRP_ERR_DEVICE, CRP_ERR_UNSUPPORTED, CRP_ERR_WORKSPACE = 0, -1, -2, -3, -4
CRP_F64, CRP_F32, CRP_F16, CRP_BF16 = 0, 1, 2, 3
CRP_LAYOUT_LINEAR, CRP_LAYOUT_CELL8 = 0, 1
CRP_PREC_FP64, CRP_PREC_MIXED_F64ACC, CRP_PREC_MIXED_DFACC = 0, 1, 2
STATUS = {"ACTIVE": 0, "ARRIVED": 1, "MAX_LENGTH": 2, "MAX_STEPS": 3, "NONFINITE": 4,
          "CANCELLED": 5, "BAD_INPUT": 6}
COUNTERS = ["evals", "accepted", "rejected", "event_evals", "floor_hits", "particles", "cell_loads", "wave_iters"]
NCOUNTERS = 8
DTYPES = {"f64": CRP_F64, "f32": CRP_F32, "f16": CRP_F16, "bf16": CRP_BF16}
LAYOUTS = {"linear": CRP_LAYOUT_LINEAR, "cell8": CRP_LAYOUT_CELL8}


class CRPError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"libcrp status {status}: {message}")
        self.status = status


class crp_modulation(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("dtype", C.c_int32), ("origin", C.c_double * 3), ("spacing", C.c_double),
                ("data", C.c_void_p)]


class crp_field(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("dtype", C.c_int32), ("layout", C.c_int32),
                ("reserved", C.c_int32), ("origin", C.c_double * 3), ("spacing", C.c_double),
                ("value_scale", C.c_double), ("data", C.c_void_p), ("modulation", C.POINTER(crp_modulation))]


class crp_params(C.Structure):
    _fields_ = [("tol", C.c_double), ("h_min", C.c_double), ("h_max", C.c_double),
                ("obs_center", C.c_double * 3), ("obs_radius", C.c_double), ("l_max", C.c_double),
                ("max_steps", C.c_int64), ("field_index", C.c_int32), ("reflect", C.c_int32),
                ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3), ("backtrack", C.c_int32),
                ("reserved", C.c_int32)]


_PARTICLE_FIELDS = ["x", "y", "z", "ux", "uy", "uz", "energy", "charge", "mass", "length",
                    "h_next", "time", "status", "param_index", "n_accepted", "n_rejected"]


class crp_particles(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in _PARTICLE_FIELDS]


class crp_tape(C.Structure):
    _fields_ = [("checkpoints", C.c_void_p), ("links", C.c_void_p), ("head", C.c_void_p), ("finals", C.c_void_p),
                ("capacity", C.c_int64), ("every_k", C.c_int32), ("reserved", C.c_int32)]


CRP_TAPE_EVENT, CRP_TAPE_OVERFLOW, CRP_TAPE_FRESH, CRP_TAPE_COMPLETE = 1, 2, 4, 8
CRP_TAPE_MIRRORED, CRP_TAPE_GRAD_OVERFLOW = 16, 32


class crp_tuning(C.Structure):
    _fields_ = [("block_size", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("refill_threshold", C.c_int32), ("order_by_rigidity", C.c_int32),
                ("cache_cells", C.c_int32), ("reserved", C.c_int32), ("cancel", C.c_void_p)]


_lib = None


def lib():
    """Load libcrp.so from the package directory (raises if absent)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libcrp.so not built at {LIB_PATH}; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        L.crp_field_bytes.argtypes = [C.POINTER(crp_field)]
        L.crp_field_bytes.restype = C.c_size_t
        L.crp_field_upload.argtypes = [C.POINTER(crp_field), C.c_void_p, C.c_int32, C.c_void_p]
        L.crp_modulation_bytes.argtypes = [C.POINTER(crp_modulation)]
        L.crp_modulation_bytes.restype = C.c_size_t
        L.crp_modulation_upload.argtypes = [C.POINTER(crp_modulation), C.c_void_p, C.c_int32, C.c_void_p]
        L.crp_modulation_upload.restype = C.c_int
        L.crp_workspace_bytes.argtypes = [C.c_int64, C.c_int32, C.c_int32]
        L.crp_workspace_bytes.restype = C.c_size_t
        L.crp_propagate.argtypes = [C.POINTER(crp_field), C.c_int32, C.POINTER(crp_params), C.c_int32,
                                    C.POINTER(crp_particles), C.c_int64, C.POINTER(crp_tape), C.c_int32,
                                    C.POINTER(crp_tuning), C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
        L.crp_propagate_noalloc.argtypes = [C.POINTER(crp_field), C.c_int32, C.POINTER(crp_params), C.c_int32,
                                            C.POINTER(crp_particles), C.c_int64, C.POINTER(crp_tape), C.c_int32,
                                            C.POINTER(crp_tuning), C.c_void_p, C.c_void_p]
        L.crp_propagate_noalloc.restype = C.c_int
        L.crp_noalloc_scratch_bytes.argtypes = []
        L.crp_noalloc_scratch_bytes.restype = C.c_size_t
        L.crp_adjoint_workspace_bytes.argtypes = [C.c_int64, C.c_int32]
        L.crp_adjoint_workspace_bytes.restype = C.c_size_t
        L.crp_adjoint_replay_workspace_bytes.argtypes = [C.c_int64, C.c_int32, C.c_int64]
        L.crp_adjoint_replay_workspace_bytes.restype = C.c_size_t
        L.crp_propagate_adjoint.argtypes = [C.POINTER(crp_field), C.POINTER(crp_params), C.POINTER(crp_particles),
                                            C.c_int64, C.POINTER(crp_tape), C.c_void_p, C.c_void_p, C.c_void_p,
                                            C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                            C.c_void_p, C.c_size_t, C.c_void_p]
        L.crp_propagate_adjoint.restype = C.c_int
        L.crp_selftest_arith.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p]
        L.crp_bench_gather.argtypes = [C.POINTER(crp_field), C.c_int64, C.c_int64, C.c_double, C.c_uint64,
                                       C.c_void_p, C.c_void_p]
        L.crp_bench_stream.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p, C.c_int32, C.c_void_p]
        L.crp_bench_gather.restype = C.c_int
        L.crp_bench_gather_replay.argtypes = [C.POINTER(crp_field), C.c_void_p, C.c_int64, C.c_int64, C.c_int32,
                                              C.c_void_p, C.c_void_p, C.c_void_p]
        L.crp_bench_gather_replay.restype = C.c_int
        L.crp_bench_stream.restype = C.c_int
        L.crp_graph_create.argtypes = [C.POINTER(crp_field), C.c_int32, C.POINTER(crp_params), C.c_int32,
                                       C.POINTER(crp_particles), C.c_int64, C.c_int32, C.POINTER(crp_tuning),
                                       C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]
        L.crp_graph_launch.argtypes = [C.c_void_p, C.c_void_p]
        L.crp_graph_destroy.argtypes = [C.c_void_p]
        for f in (L.crp_graph_create, L.crp_graph_launch, L.crp_graph_destroy):
            f.restype = C.c_int
        L.crp_healpix_pixels.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                         C.c_void_p]
        L.crp_lens_workspace_bytes.argtypes = [C.c_int32, C.c_int64]
        L.crp_lens_workspace_bytes.restype = C.c_size_t
        L.crp_lens_build.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                     C.POINTER(C.c_int64), C.c_void_p, C.c_size_t, C.c_void_p]
        L.crp_lens_apply.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                     C.c_void_p, C.c_int32, C.c_void_p]
        for f in (L.crp_healpix_pixels, L.crp_lens_build, L.crp_lens_apply):
            f.restype = C.c_int
        L.crp_last_error.restype = C.c_char_p
        L.crp_version.restype = C.c_char_p
        for f in (L.crp_field_upload, L.crp_propagate, L.crp_selftest_arith):
            f.restype = C.c_int
        _lib = L
    return _lib


def _check(status: int):
    if status != CRP_OK:
        raise CRPError(status, lib().crp_last_error().decode())


def _torch():
    import torch
    return torch


def _stream_handle(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


# ---------------------------------------------------------------- entry points

def crp_version() -> str:
    return lib().crp_version().decode()


def crp_last_error() -> str:
    return lib().crp_last_error().decode()


def crp_field_bytes(desc: crp_field) -> int:
    return int(lib().crp_field_bytes(C.byref(desc)))


def crp_workspace_bytes(n: int, n_fields: int = 1, n_params: int = 1) -> int:
    return int(lib().crp_workspace_bytes(int(n), int(n_fields), int(n_params)))


def crp_field_upload(desc: crp_field, src, stream=None):
    """src: CUDA tensor float64/float32 of shape (n0, n1, n2, 3), nG."""
    torch = _torch()
    if src.dtype == torch.float64:
        sd = CRP_F64
    elif src.dtype == torch.float32:
        sd = CRP_F32
    else:
        raise TypeError("source grid must be float64 or float32")
    if not src.is_contiguous() or not src.is_cuda:
        raise ValueError("source grid must be a contiguous device tensor")
    if tuple(src.shape) != (desc.n[0], desc.n[1], desc.n[2], 3):
        raise ValueError(f"source shape {tuple(src.shape)} does not match the descriptor")
    _check(lib().crp_field_upload(C.byref(desc), _ptr(src), sd, _stream_handle(stream)))


class Tape:
    """Device tape of a forward run: a pool of `capacity` checkpoint records,
    taken every `every_k` accepted steps, plus per-particle finals."""

    def __init__(self, n: int, every_k: int = 64, capacity: int | None = None, device="cuda"):
        torch = _torch()
        n = int(n)
        self.capacity = int(capacity) if capacity is not None else 64 * n + 1024
        if self.capacity < 1:
            raise ValueError("a tape needs at least one record")
        self.checkpoints = torch.empty(self.capacity * 8, dtype=torch.float64, device=device)
        self.links = torch.empty(self.capacity, dtype=torch.int64, device=device)
        self.head = torch.zeros(1, dtype=torch.int64, device=device)
        self.finals = torch.zeros(4 * n, dtype=torch.float64, device=device)
        self.every_k = int(every_k)
        self.desc = crp_tape(self.checkpoints.data_ptr(), self.links.data_ptr(), self.head.data_ptr(),
                             self.finals.data_ptr(), self.capacity, self.every_k, 0)

    def reset(self):
        """Zero the pool head before recording another run into this tape."""
        self.head.zero_()

    def records_needed(self) -> int:
        """Records the last run asked for (more than capacity after an overflow)."""
        return int(self.head.item())

    def overflowed(self) -> bool:
        return self.records_needed() > self.capacity

    def flags(self):
        return self.finals.view(-1, 4)[:, 3].to(_torch().int32)

    def steps(self):
        return self.finals.view(-1, 4)[:, 0].to(_torch().int64)

    def replay_steps(self, fraction: float = 0.5) -> int:
        """Parallel-replay room (in records) for the particles that took at
        least `fraction` of the most steps any particle took, which takes their
        replay off the adjoint's critical path.  The adjoint replays groups of
        64 consecutive particles of its order, each group padded to its most
        steps; the order sorts by steps only within buckets of 1/8 in log2, so
        the padded size is estimated on the sorted steps with a 10% margin."""
        torch = _torch()
        N = self.steps()
        if N.numel() == 0:
            return 0
        top = int(N.max().item())
        if top <= 0:
            return 0
        keep = torch.sort(N[N >= max(1, int(fraction * top))], descending=True).values
        pad = (-keep.numel()) % 64
        keep = torch.cat([keep, keep.new_zeros(pad)]).view(-1, 64)
        return int(1.1 * 64 * int(keep.max(dim=1).values.sum().item())) + 64

    @property
    def nbytes(self) -> int:
        return self.capacity * 72 + self.finals.numel() * 8 + 8


def crp_propagate(fields, params, particles: dict, precision=CRP_PREC_FP64, tuning=None,
                  counters=None, workspace=None, stream=None, tape=None):
    """Propagate in place.  fields: list of Field; params: list of crp_params;
    particles: dict of device tensors keyed as in crp_particles; tape: a Tape."""
    torch = _torch()
    farr, nf, parr, np_, ps, n, tun = _marshal(fields, params, particles, tuning)
    need = crp_workspace_bytes(n, nf, np_)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=particles["energy"].device)
    _check(lib().crp_propagate(farr, nf, parr, np_, C.byref(ps), n, C.byref(tape.desc) if tape else None,
                               int(precision), tun, _ptr(counters), _ptr(workspace), workspace.numel(),
                               _stream_handle(stream)))
    return particles


def crp_propagate_noalloc(fields, params, particles: dict, precision=CRP_PREC_FP64, tuning=None,
                          counters=None, stream=None, tape=None):
    """crp_propagate without a workspace: the library's per-GPU scratch array
    is used instead (for callers that cannot allocate device memory)."""
    farr, nf, parr, np_, ps, n, tun = _marshal(fields, params, particles, tuning)
    _check(lib().crp_propagate_noalloc(farr, nf, parr, np_, C.byref(ps), n, C.byref(tape.desc) if tape else None,
                                       int(precision), tun, _ptr(counters), _stream_handle(stream)))
    return particles


def crp_noalloc_scratch_bytes() -> int:
    return int(lib().crp_noalloc_scratch_bytes())


def crp_adjoint_workspace_bytes(n: int, every_k: int) -> int:
    return int(lib().crp_adjoint_workspace_bytes(int(n), int(every_k)))


def crp_adjoint_replay_workspace_bytes(n: int, every_k: int, replay_steps: int) -> int:
    return int(lib().crp_adjoint_replay_workspace_bytes(int(n), int(every_k), int(replay_steps)))


def adjoint_workspace(n: int, tape: Tape, replay_steps="auto", device="cuda"):
    """Workspace for crp_propagate_adjoint.  replay_steps: room for parallel
    replay, in accepted steps; "auto" sizes it with tape.replay_steps() (after
    the taped run) within a quarter of the free device memory; 0: none."""
    torch = _torch()
    if replay_steps == "auto":
        replay_steps = tape.replay_steps()
        free = torch.cuda.mem_get_info(torch.device(device))[0]
        base = crp_adjoint_workspace_bytes(n, tape.every_k)
        while replay_steps > 0 and crp_adjoint_replay_workspace_bytes(n, tape.every_k, replay_steps) - base > free // 4:
            replay_steps //= 2
    nbytes = crp_adjoint_replay_workspace_bytes(n, tape.every_k, int(replay_steps))
    if nbytes == 0:
        raise ValueError("invalid adjoint workspace arguments")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def crp_propagate_adjoint(field, params, initial: dict, tape: Tape, gbar_dir, gbar_time, grad_u0, grad_field,
                          grad_x0=None, gbar_energy=None, workspace=None, stream=None, grad_energy=None,
                          replay_steps="auto"):
    """Reverse-mode derivatives of a taped forward run (see crp.h).  Without a
    workspace, one is allocated with adjoint_workspace(n, tape, replay_steps).
    grad_field: a float64 or float32 tensor (the grid gradient's dtype)."""
    torch = _torch()
    if grad_field.dtype not in (torch.float64, torch.float32):
        raise TypeError("grad_field must be float64 or float32")
    gdt = CRP_F64 if grad_field.dtype == torch.float64 else CRP_F32
    n = int(initial["energy"].numel())
    ps = crp_particles(**{k: (initial[k].data_ptr() if initial.get(k) is not None else None)
                          for k in _PARTICLE_FIELDS})
    if workspace is None:
        workspace = adjoint_workspace(n, tape, replay_steps, device=initial["energy"].device)
    _check(lib().crp_propagate_adjoint(C.byref(field.desc), C.byref(params), C.byref(ps), n, C.byref(tape.desc),
                                       _ptr(gbar_dir), _ptr(gbar_time), _ptr(gbar_energy), _ptr(grad_u0),
                                       _ptr(grad_x0), _ptr(grad_energy), _ptr(grad_field), gdt, _ptr(workspace),
                                       workspace.numel(),
                                       _stream_handle(stream)))


def healpix_npix(nside: int) -> int:
    return 12 * int(nside) * int(nside)


def crp_healpix_pixels(nside: int, ux, uy, uz, pix=None, stream=None):
    """RING-scheme HEALPix pixel (int32, -1 for a zero direction) of each direction."""
    torch = _torch()
    n = int(ux.numel())
    if pix is None:
        pix = torch.empty(n, dtype=torch.int32, device=ux.device)
    _check(lib().crp_healpix_pixels(int(nside), _ptr(ux), _ptr(uy), _ptr(uz), n, _ptr(pix),
                                    _stream_handle(stream)))
    return pix


def crp_lens_workspace_bytes(nside: int, n: int) -> int:
    return int(lib().crp_lens_workspace_bytes(int(nside), int(n)))


class Lens:
    """A CSR lens over HEALPix pixels (device tensors) for one rigidity."""

    def __init__(self, nside, row_ptr, col, val, nnz):
        self.nside, self.row_ptr, self.nnz = int(nside), row_ptr, int(nnz)
        self.col, self.val = col[:self.nnz], val[:self.nnz]

    @property
    def npix(self) -> int:
        return healpix_npix(self.nside)

    def nbytes(self) -> int:
        return 8 * (self.npix + 1) + 8 * self.nnz


def crp_lens_build(nside: int, rows, particles: dict, workspace=None, stream=None, out=None) -> Lens:
    """Lens from the launches' observed pixels (rows) and the output of their
    backtracking run (particles: ux, uy, uz, status).  Waits for the stream.
    out: optional (row_ptr, col, val) device tensors to write into."""
    torch = _torch()
    n = int(rows.numel())
    dev = rows.device
    npx = healpix_npix(nside)
    if out is not None:
        row_ptr, col, val = out
    else:
        row_ptr = torch.empty(npx + 1, dtype=torch.int64, device=dev)
        col = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        val = torch.empty(max(n, 1), dtype=torch.float32, device=dev)
    if workspace is None:
        workspace = torch.empty(crp_lens_workspace_bytes(nside, n), dtype=torch.uint8, device=dev)
    nnz = C.c_int64(0)
    _check(lib().crp_lens_build(int(nside), _ptr(rows), _ptr(particles["ux"]), _ptr(particles["uy"]),
                                _ptr(particles["uz"]), _ptr(particles["status"]), n, _ptr(row_ptr), _ptr(col),
                                _ptr(val), col.numel(), C.byref(nnz), _ptr(workspace), workspace.numel(),
                                _stream_handle(stream)))
    return Lens(nside, row_ptr, col, val, nnz.value)


def crp_lens_apply(lens: Lens, x, y=None, stream=None):
    """y = L x for x of shape (npix,) or (npix, nvec), float32 on the device."""
    torch = _torch()
    x = x.contiguous()
    nvec = 1 if x.dim() == 1 else int(x.shape[1])
    if y is None:
        y = torch.empty_like(x)
    _check(lib().crp_lens_apply(lens.nside, _ptr(lens.row_ptr), _ptr(lens.col), _ptr(lens.val), lens.nnz, _ptr(x),
                                _ptr(y), nvec, _stream_handle(stream)))
    return y


def _marshal(fields, params, particles, tuning):
    nf, np_ = len(fields), len(params)
    farr = (crp_field * nf)(*[f.desc for f in fields])
    parr = (crp_params * np_)(*params)
    n = int(particles["energy"].numel())
    ps = crp_particles(**{k: (particles[k].data_ptr() if particles.get(k) is not None else None)
                          for k in _PARTICLE_FIELDS})
    tun = C.byref(tuning) if tuning is not None else None
    return farr, nf, parr, np_, ps, n, tun


class Graph:
    """A captured crp_propagate (crp_graph_create); replay with launch().

    The captured pointers (fields, particles, workspace, counters) are kept
    alive by this object.  Capture and replay run on a dedicated stream that
    is ordered after the caller's current stream."""

    def __init__(self, fields, params, particles: dict, precision=CRP_PREC_FP64, tuning=None, counters=None,
                 workspace=None):
        torch = _torch()
        self._keep = (fields, params, particles, counters, tuning)
        farr, nf, parr, np_, ps, n, tun = _marshal(fields, params, particles, tuning)
        self._arrays = (farr, parr, ps)
        dev = particles["energy"].device
        self.workspace = workspace if workspace is not None else \
            torch.empty(crp_workspace_bytes(n, nf, np_), dtype=torch.uint8, device=dev)
        self.stream = torch.cuda.Stream(device=dev)
        self.stream.wait_stream(torch.cuda.current_stream(dev))
        h = C.c_void_p()
        _check(lib().crp_graph_create(farr, nf, parr, np_, C.byref(ps), n, int(precision), tun, _ptr(counters),
                                      _ptr(self.workspace), self.workspace.numel(),
                                      C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.handle = h

    def launch(self):
        torch = _torch()
        cur = torch.cuda.current_stream(self.stream.device)
        self.stream.wait_stream(cur)
        _check(lib().crp_graph_launch(self.handle, C.c_void_p(self.stream.cuda_stream)))
        cur.wait_stream(self.stream)

    def close(self):
        if self.handle:
            self.stream.synchronize()
            _check(lib().crp_graph_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def crp_selftest_arith(inp, out, op: int, stream=None):
    n = out.numel()
    _check(lib().crp_selftest_arith(_ptr(inp), _ptr(out), n, int(op), _stream_handle(stream)))


def crp_bench_gather(field, lanes: int, lookups_per_lane: int, spread: float, seed: int, sink, stream=None):
    _check(lib().crp_bench_gather(C.byref(field.desc), int(lanes), int(lookups_per_lane), float(spread),
                                  int(seed), _ptr(sink), _stream_handle(stream)))


def crp_bench_gather_replay(field, rec, lanes: int, steps: int, cache: bool, sink, misses=None, stream=None):
    _check(lib().crp_bench_gather_replay(C.byref(field.desc), _ptr(rec), int(lanes), int(steps), 1 if cache else 0,
                                         _ptr(sink), _ptr(misses), _stream_handle(stream)))


def crp_bench_stream(src, dst, nbytes: int, sink, blocks: int, stream=None):
    _check(lib().crp_bench_stream(_ptr(src), _ptr(dst), int(nbytes), _ptr(sink), int(blocks),
                                  _stream_handle(stream)))


# ------------------------------------------------------------- conveniences

@dataclass
class Modulation:
    """A device modulation grid: descriptor plus the tensor that owns its storage."""
    desc: crp_modulation
    storage: object


def make_modulation(values, spacing: float, origin=(0.0, 0.0, 0.0), dtype="f32", device="cuda",
                    stream=None) -> Modulation:
    """Upload an (n0, n1, n2) scalar modulation grid (numpy or torch; float64/float32)."""
    torch = _torch()
    src = values if isinstance(values, torch.Tensor) else torch.from_numpy(values)
    src = src.to(device=device).contiguous()
    if src.dtype not in (torch.float64, torch.float32) or src.dim() != 3:
        raise TypeError("modulation must be a float64/float32 array of shape (n0, n1, n2)")
    d = crp_modulation()
    d.n[0], d.n[1], d.n[2] = (int(v) for v in src.shape)
    d.dtype = DTYPES[dtype]
    d.origin[0], d.origin[1], d.origin[2] = (float(o) for o in origin)
    d.spacing = float(spacing)
    nb = int(lib().crp_modulation_bytes(C.byref(d)))
    if nb == 0:
        raise CRPError(CRP_ERR_INVALID, crp_last_error())
    storage = torch.empty(nb, dtype=torch.uint8, device=device)
    d.data = storage.data_ptr()
    sd = CRP_F64 if src.dtype == torch.float64 else CRP_F32
    _check(lib().crp_modulation_upload(C.byref(d), _ptr(src), sd, _stream_handle(stream)))
    torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    return Modulation(d, storage)


@dataclass
class Field:
    """A device field grid: descriptor plus the torch tensor that owns its storage
    (and the modulation it refers to, if any)."""
    desc: crp_field
    storage: object
    modulation: object = None

    @property
    def nbytes(self) -> int:
        return crp_field_bytes(self.desc)


def make_field(values, spacing: float, origin=(0.0, 0.0, 0.0), dtype="f32", layout="linear",
               value_scale: float = 1.0, device="cuda", stream=None, modulation: Modulation | None = None) -> Field:
    """Upload an (n0, n1, n2, 3) grid in nG (numpy or torch; float64/float32),
    optionally multiplied by a Modulation (section 3.2, modulated grids)."""
    torch = _torch()
    src = values if isinstance(values, torch.Tensor) else torch.from_numpy(values)
    src = src.to(device=device).contiguous()
    d = crp_field()
    d.n[0], d.n[1], d.n[2] = (int(s) for s in src.shape[:3])
    d.dtype = DTYPES[dtype]
    d.layout = LAYOUTS[layout]
    d.origin[0], d.origin[1], d.origin[2] = (float(o) for o in origin)
    d.spacing = float(spacing)
    d.value_scale = float(value_scale)
    nb = crp_field_bytes(d)
    if nb == 0:
        raise CRPError(CRP_ERR_INVALID, crp_last_error())
    storage = torch.empty(nb, dtype=torch.uint8, device=device)
    d.data = storage.data_ptr()
    crp_field_upload(d, src, stream=stream)
    torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    if modulation is not None:
        d.modulation = C.pointer(modulation.desc)
    return Field(d, storage, modulation)


def make_params(tol, h_min, h_max, obs_radius=0.0, l_max=math.inf, obs_center=(0.0, 0.0, 0.0),
                max_steps=0, field_index=0, box=None, backtrack=False) -> crp_params:
    """One parameter group; ``box`` = ((lo x, y, z), (hi x, y, z)) in Mpc turns on
    the reflective box; ``backtrack`` traces the
    particles back from where they were observed."""
    p = crp_params()
    p.backtrack = 1 if backtrack else 0
    if box is not None:
        p.reflect = 1
        for i in range(3):
            p.box_lo[i], p.box_hi[i] = float(box[0][i]), float(box[1][i])
    p.tol, p.h_min, p.h_max = float(tol), float(h_min), float(h_max)
    for i in range(3):
        p.obs_center[i] = float(obs_center[i])
    p.obs_radius = float(obs_radius)
    p.l_max = float(l_max)
    p.max_steps = int(max_steps)
    p.field_index = int(field_index)
    return p


def make_tuning(block_size=256, blocks_per_cu=4, refill_threshold=32, order_by_rigidity=1,
                cache_cells=0, cancel=None) -> crp_tuning:
    """Launch configuration; ``cancel`` is an optional device int32 tensor (one
    element) whose becoming nonzero stops the call early (resumable)."""
    return crp_tuning(block_size, blocks_per_cu, refill_threshold, order_by_rigidity, cache_cells, 0,
                      None if cancel is None else cancel.data_ptr())


def particles_to_device(pos, dir, energy, charge, mass=None, param_index=None, device="cuda",
                        with_time=True) -> dict:
    """Copy host particle arrays into the SoA device tensors of crp_particles (fresh start)."""
    torch = _torch()
    import numpy as np
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    dir = np.asarray(dir, dtype=np.float64).reshape(-1, 3)
    n = pos.shape[0]

    def d64(a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(device)

    def i32(a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(device)

    p = {"x": d64(pos[:, 0]), "y": d64(pos[:, 1]), "z": d64(pos[:, 2]),
         "ux": d64(dir[:, 0]), "uy": d64(dir[:, 1]), "uz": d64(dir[:, 2]),
         "energy": d64(energy), "charge": i32(charge),
         "mass": i32(mass) if mass is not None else None,
         "length": torch.zeros(n, dtype=torch.float64, device=device),
         "h_next": torch.zeros(n, dtype=torch.float64, device=device),
         "time": torch.zeros(n, dtype=torch.float64, device=device) if with_time else None,
         "status": torch.zeros(n, dtype=torch.int32, device=device),
         "param_index": i32(param_index) if param_index is not None else None,
         "n_accepted": torch.zeros(n, dtype=torch.int64, device=device),
         "n_rejected": torch.zeros(n, dtype=torch.int64, device=device)}
    return p


def particles_to_host(p: dict) -> dict:
    """Gather device particle state into numpy arrays (pos/dir as (n, 3))."""
    import numpy as np
    out = {k: v.cpu().numpy() for k, v in p.items() if v is not None}
    out["pos"] = np.stack([out.pop("x"), out.pop("y"), out.pop("z")], axis=1)
    out["dir"] = np.stack([out.pop("ux"), out.pop("uy"), out.pop("uz")], axis=1)
    return out


def clone_particles(p: dict) -> dict:
    return {k: (v.clone() if v is not None else None) for k, v in p.items()}
