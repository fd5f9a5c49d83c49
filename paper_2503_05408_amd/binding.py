"""ctypes binding of ``libgltrsv.so`` (declared in ``include/gltrsv.h``).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels, and the scheduling/packing in its host C++.  PyTorch provides device
memory and streams.  If the library cannot be loaded the calls raise; there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

from . import build as _build

_lock = threading.Lock()
_lib = None

P = ctypes.c_void_p
i32, i64, u64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double

GLTRSV_OK = 0
ERRORS = {
    -1: "EINVAL", -2: "ENOTLOWER", -3: "ESINGULAR", -4: "EUNSORTED", -5: "ERANGE",
    -6: "ENOMEM", -7: "EAGAIN", -8: "EHIP", -9: "ETIMEDOUT", -10: "ENOTSUP", -11: "ENOENT",
}
SCHED_GROWLOCAL = 0
SCHED_WAVEFRONT = 1
SCHED_AUTO = 2
SCHED_GIVEN = 3
LOWER = 0
UPPER = 1
PACK_AUTO = 0
PACK_HOST = 1
PACK_DEVICE = 2
EXEC_PERSISTENT = 0
EXEC_PLAIN = 1
EXEC_ASYNC = 2
EXEC_LOCAL = 3
EXEC_FORMS = 4
EXEC_NAMES = {EXEC_PERSISTENT: "persistent", EXEC_PLAIN: "plain", EXEC_ASYNC: "async", EXEC_LOCAL: "local"}


class GltrsvError(RuntimeError):
    def __init__(self, code: int, where: str, text: str):
        super().__init__(f"{where}: {ERRORS.get(code, code)} ({text})")
        self.code = code


class Csr(ctypes.Structure):
    _fields_ = [("n", i64), ("nnz", i64), ("row_ptr", P), ("col", P), ("val", P)]


class PlanOpts(ctypes.Structure):
    _fields_ = [("k", i32), ("L", dbl), ("alpha0", dbl), ("growth", dbl), ("accept", dbl),
                ("schedule_kind", i32), ("reorder", i32), ("block_size", i32), ("grid_blocks", i32),
                ("cooperative", i32), ("analysis_threads", i32), ("pack", i32),
                ("blocks", i32), ("triangle", i32), ("funnel_max_weight", i32),
                ("exec_hint", i32), ("core_width", i32)]


class BatchOpts(ctypes.Structure):
    _fields_ = [("per_claim", i32), ("grid_blocks", i32), ("use_graph", i32), ("async_exec", i32)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("budget_bytes", i64), ("max_slots", i32), ("per_claim", i32), ("quantum_us", dbl),
                ("counter_words", i32), ("grid_blocks", i32), ("async_exec", i32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", i64), ("completed", i64), ("failed", i64), ("launches", i64),
                ("rows_completed", i64), ("queued", i64), ("inflight_bytes", i64), ("cancelled", i64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class PlanInfo(ctypes.Structure):
    _fields_ = [("n", i64), ("nnz", i64), ("supersteps", i32), ("wavefronts", i32), ("tasks", i64),
                ("chunks", i64), ("stream_slots", i64), ("device_bytes", i64), ("analysis_ns", i64),
                ("pattern_key", u64), ("grid_blocks", i32), ("block_size", i32), ("max_task_rows", i64),
                ("schedule_kind", i32), ("predicted_us", dbl), ("device_packed", i32),
                ("async_grid_blocks", i32), ("exec_form", i32), ("core_width", i32),
                ("local_groups", i64), ("local_records", i64), ("local_far", i64),
                ("row_dpp", i32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


# function name -> (argtypes, restype)
SIGNATURES = {
    "gltrsv_last_error": ([], ctypes.c_char_p),
    "gltrsv_version": ([], ctypes.c_char_p),
    "gltrsv_check_csr": ([P], i32),
    "gltrsv_default_opts": ([P], None),
    "gltrsv_levels": ([P, P, P], i32),
    "gltrsv_schedule": ([P, P, P, P, P], i32),
    "gltrsv_reorder": ([i64, P, P, P], i32),
    "gltrsv_plan_create": ([P, P, P], i32),
    "gltrsv_plan_create_with_schedule": ([P, P, P, P, P], i32),
    "gltrsv_plan_info_get": ([P, P], i32),
    "gltrsv_plan_schedule": ([P, P, P, P], i32),
    "gltrsv_plan_destroy": ([P], i32),
    "gltrsv_solve": ([P, P, P, P], i32),
    "gltrsv_solve_plain": ([P, P, P, P], i32),
    "gltrsv_plan_device_status": ([P, P], i32),
    "gltrsv_debug_trace": ([P, P, i64], i32),
    "gltrsv_copy_probe": ([P, P, i64, P], i32),
    "gltrsv_plan_gather_probe": ([P, P, P, P], i32),
    "gltrsv_solve_async": ([P, P, P, P], i32),
    "gltrsv_solve_local": ([P, P, P, P], i32),
    "gltrsv_plan_local_size": ([P, P, P], i32),
    "gltrsv_plan_local_records": ([P, P, i64, P, i64], i32),
    "gltrsv_local_layout": ([P, i32, P, P, P, P, P, P], i32),
    "gltrsv_wave_streams": ([P, i32, P, P, i64, P, P, P, P, P, P], i32),
    "gltrsv_solve_multi": ([P, P, P, i32, P], i32),
    "gltrsv_plan_set_spin_limit": ([P, i64], i32),
    "gltrsv_plan_set_steal_wait": ([P, i64], i32),
    "gltrsv_plan_set_start_delay": ([P, i64], i32),
    "gltrsv_solve_auto": ([P, P, P, P], i32),
    "gltrsv_solve_unordered": ([P, P, P, P], i32),
    "gltrsv_plan_set_exec": ([P, i32], i32),
    "gltrsv_plan_tune": ([P, P, P, i32, P, P, P], i32),
    "gltrsv_plan_stream": ([P, P, P, i64], i32),
    "gltrsv_default_batch_opts": ([P], None),
    "gltrsv_batch_create": ([P, i32, P, P], i32),
    "gltrsv_batch_solve": ([P, P, P, P], i32),
    "gltrsv_batch_status": ([P, P], i32),
    "gltrsv_batch_info": ([P, P, P], i32),
    "gltrsv_batch_destroy": ([P], i32),
    "gltrsv_solve_batched": ([P, P, P, i32, P], i32),
    "gltrsv_solve_batched_noalloc": ([P, P, P, i32, P], i32),
    "gltrsv_default_server_opts": ([P], None),
    "gltrsv_server_create": ([P, P], i32),
    "gltrsv_server_submit": ([P, P, P, P, P], i32),
    "gltrsv_server_poll": ([P, P, P, i32, P], i32),
    "gltrsv_server_get_stats": ([P, P], i32),
    "gltrsv_server_cancel": ([P, u64], i32),
    "gltrsv_clock_ns": ([], i64),
    "gltrsv_server_destroy": ([P], i32),
}


def lib_path() -> str:
    return _build.LIB


def load(build_if_missing: bool = True):
    """Loads the HIP library (building it only if no build exists).

    torch is imported first: its wheel carries its own HIP runtime, and the
    library must bind to that same runtime (loading the library first would
    bring a second runtime into the process, and the one initialised second
    finds no device)."""
    global _lib
    with _lock:
        if _lib is None:
            import torch  # noqa: F401
            if not os.path.exists(_build.LIB):
                if not build_if_missing:
                    raise RuntimeError(f"{_build.LIB} is not built")
                _build.build()
            lib = ctypes.CDLL(_build.LIB)
            for name, (argt, rest) in SIGNATURES.items():
                f = getattr(lib, name)
                f.argtypes = argt
                f.restype = rest
            _lib = lib
    return _lib


def _check(rc: int, where: str):
    if rc != GLTRSV_OK:
        raise GltrsvError(rc, where, load().gltrsv_last_error().decode())


def _np_ptr(a):
    return a.ctypes.data_as(P)


class _HostCsr:
    """Keeps numpy arrays alive while a Csr struct points at them."""

    def __init__(self, m):
        self.rp = np.ascontiguousarray(m.row_ptr, dtype=np.int64)
        self.col = np.ascontiguousarray(m.col, dtype=np.int32)
        self.val = None if m.val is None else np.ascontiguousarray(m.val, dtype=np.float64)
        self.s = Csr(int(m.n), int(self.rp[-1]) if self.rp.size else 0, _np_ptr(self.rp), _np_ptr(self.col),
                     None if self.val is None else _np_ptr(self.val))

    @property
    def ref(self):
        return ctypes.byref(self.s)


def default_opts(**overrides) -> PlanOpts:
    o = PlanOpts()
    load().gltrsv_default_opts(ctypes.byref(o))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def gpu_opts(**overrides) -> PlanOpts:
    """Schedule parameters sized for the GPU: many lane-cores, a barrier cost
    L expressed in the weight units of one lane, and alpha starting at 1."""
    base = dict(k=1 << 16, L=50.0, alpha0=1.0)
    base.update(overrides)
    return default_opts(**base)


def check_csr(m) -> int:
    h = _HostCsr(m)
    return int(load().gltrsv_check_csr(h.ref))


def levels(m):
    h = _HostCsr(m)
    lv = np.empty(m.n, dtype=np.int32)
    nl = ctypes.c_int32(0)
    _check(load().gltrsv_levels(h.ref, _np_ptr(lv), ctypes.byref(nl)), "gltrsv_levels")
    return lv, nl.value


def schedule(m, opts: PlanOpts | None = None):
    h = _HostCsr(m)
    opts = opts or default_opts()
    core = np.empty(m.n, dtype=np.int32)
    sup = np.empty(m.n, dtype=np.int32)
    S = ctypes.c_int32(0)
    _check(load().gltrsv_schedule(h.ref, ctypes.byref(opts), _np_ptr(core), _np_ptr(sup), ctypes.byref(S)),
           "gltrsv_schedule")
    return core, sup, S.value


def wave_streams(m, core, superstep, waves: int, triangle: int = 0):
    """Host-built per-wave record streams of the schedule (core, superstep)
    per row for `waves` waves: dict of scol (uint32), sval (float64), sbeg
    (int64 [waves + 1]) and stask (int64 [tasks])."""
    h = _HostCsr(m)
    core = np.ascontiguousarray(core, dtype=np.int32)
    superstep = np.ascontiguousarray(superstep, dtype=np.int32)
    ns, nt = ctypes.c_int64(0), ctypes.c_int64(0)
    f = load().gltrsv_wave_streams
    _check(f(h.ref, int(triangle), _np_ptr(core), _np_ptr(superstep), int(waves), None, None, None, None,
             ctypes.byref(ns), ctypes.byref(nt)), "gltrsv_wave_streams")
    scol = np.empty(max(1, ns.value), dtype=np.uint32)
    sval = np.empty(max(1, ns.value), dtype=np.float64)
    sbeg = np.empty(int(waves) + 1, dtype=np.int64)
    stask = np.empty(max(1, nt.value), dtype=np.int64)
    _check(f(h.ref, int(triangle), _np_ptr(core), _np_ptr(superstep), int(waves), _np_ptr(scol), _np_ptr(sval),
             _np_ptr(sbeg), _np_ptr(stask), ctypes.byref(ns), ctypes.byref(nt)), "gltrsv_wave_streams")
    return {"scol": scol[:ns.value], "sval": sval[:ns.value], "sbeg": sbeg, "stask": stask[:nt.value]}


def local_layout(m, core, superstep, triangle: int = 0):
    """Host-built one-workgroup layout of the schedule (core, superstep) per
    row: (records as uint8, info as uint32 [records, 4])."""
    h = _HostCsr(m)
    core = np.ascontiguousarray(core, dtype=np.int32)
    superstep = np.ascontiguousarray(superstep, dtype=np.int32)
    nb, nr = i64(0), i64(0)
    _check(load().gltrsv_local_layout(h.ref, int(triangle), _np_ptr(core), _np_ptr(superstep), None,
                                      ctypes.byref(nb), None, ctypes.byref(nr)), "gltrsv_local_layout")
    rec = np.empty(max(1, nb.value), dtype=np.uint8)
    info = np.empty((max(1, nr.value), 4), dtype=np.uint32)
    _check(load().gltrsv_local_layout(h.ref, int(triangle), _np_ptr(core), _np_ptr(superstep), _np_ptr(rec),
                                      ctypes.byref(nb), _np_ptr(info), ctypes.byref(nr)), "gltrsv_local_layout")
    return rec[:nb.value], info[:nr.value]


def reorder(core, superstep):
    core = np.ascontiguousarray(core, dtype=np.int32)
    superstep = np.ascontiguousarray(superstep, dtype=np.int32)
    perm = np.empty(core.size, dtype=np.int32)
    _check(load().gltrsv_reorder(core.size, _np_ptr(core), _np_ptr(superstep), _np_ptr(perm)), "gltrsv_reorder")
    return perm


def _stream_ptr(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t, n):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError("expected a CUDA float64 tensor")
    if t.numel() != n or not t.is_contiguous():
        raise ValueError(f"expected a contiguous tensor of {n} values")
    return ctypes.c_void_p(t.data_ptr())


def copy_probe(src, dst, stream=None):
    """Device copy of src into dst (CUDA tensors of equal byte size)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes or not src.is_cuda or not dst.is_cuda:
        raise ValueError("copy_probe needs two CUDA tensors of the same size")
    _check(load().gltrsv_copy_probe(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), nbytes,
                                    _stream_ptr(stream)), "gltrsv_copy_probe")


class Plan:
    """A matrix analysed and resident on the current device."""

    def __init__(self, m, opts: PlanOpts | None = None, schedule=None):
        """schedule: optional (core, superstep) per row from an earlier
        analysis of the same pattern; the scheduler is then skipped."""
        self.n = int(m.n)
        self.opts = opts or default_opts()
        h = _HostCsr(m)
        ptr = ctypes.c_void_p()
        if schedule is None:
            _check(load().gltrsv_plan_create(h.ref, ctypes.byref(self.opts), ctypes.byref(ptr)),
                   "gltrsv_plan_create")
        else:
            core = np.ascontiguousarray(schedule[0], dtype=np.int32)
            sup = np.ascontiguousarray(schedule[1], dtype=np.int32)
            if core.shape != (self.n,) or sup.shape != (self.n,):
                raise ValueError("schedule arrays must have n entries")
            _check(load().gltrsv_plan_create_with_schedule(h.ref, ctypes.byref(self.opts), _np_ptr(core),
                                                            _np_ptr(sup), ctypes.byref(ptr)),
                   "gltrsv_plan_create_with_schedule")
        self._p = ptr

    def save_schedule(self, path: str):
        """Stores the plan's schedule (per row) with the pattern key, so a later
        process can rebuild the plan without rescheduling (load_schedule)."""
        core, sup, _ = self.schedule()
        inf = self.info()
        np.savez(path, core=core, superstep=sup, pattern_key=np.uint64(inf["pattern_key"]),
                 n=np.int64(inf["n"]), nnz=np.int64(inf["nnz"]))

    @classmethod
    def load_schedule(cls, m, path: str, opts: PlanOpts | None = None):
        """A plan for m from a schedule stored by save_schedule; the stored
        pattern key must equal m's."""
        with np.load(path, allow_pickle=False) as z:
            core, sup = z["core"], z["superstep"]
            key, n, nnz = int(z["pattern_key"]), int(z["n"]), int(z["nnz"])
        plan = cls(m, opts, schedule=(core, sup))
        if (plan.info()["pattern_key"], n, nnz) != (key, int(m.n), int(m.row_ptr[-1])):
            plan.close()
            raise ValueError("the stored schedule belongs to another sparsity pattern")
        return plan

    def close(self):
        if self._p:
            load().gltrsv_plan_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def handle(self):
        return self._p

    def info(self) -> dict:
        inf = PlanInfo()
        _check(load().gltrsv_plan_info_get(self._p, ctypes.byref(inf)), "gltrsv_plan_info_get")
        return inf.as_dict()

    def schedule(self):
        core = np.empty(self.n, dtype=np.int32)
        sup = np.empty(self.n, dtype=np.int32)
        perm = np.empty(self.n, dtype=np.int32)
        _check(load().gltrsv_plan_schedule(self._p, _np_ptr(core), _np_ptr(sup), _np_ptr(perm)),
               "gltrsv_plan_schedule")
        return core, sup, perm

    def solve(self, b, x=None, stream=None):
        """Persistent solve; returns x (allocated if not given)."""
        import torch
        if x is None:
            x = torch.empty_like(b)
        _check(load().gltrsv_solve(self._p, _dev_ptr(b, self.n), _dev_ptr(x, self.n), _stream_ptr(stream)),
               "gltrsv_solve")
        return x

    def solve_unordered(self, b, x=None, stream=None):
        """The schedule without the reorder of Sec. 5 (plan built with reorder=0)."""
        import torch
        if x is None:
            x = torch.empty_like(b)
        _check(load().gltrsv_solve_unordered(self._p, _dev_ptr(b, self.n), _dev_ptr(x, self.n), _stream_ptr(stream)),
               "gltrsv_solve_unordered")
        return x

    def solve_auto(self, b, x=None, stream=None):
        """Solve with the plan's preferred execution form (tune / set_exec)."""
        import torch
        if x is None:
            x = torch.empty_like(b)
        _check(load().gltrsv_solve_auto(self._p, _dev_ptr(b, self.n), _dev_ptr(x, self.n), _stream_ptr(stream)),
               "gltrsv_solve_auto")
        return x

    def set_exec(self, form: int):
        """Sets the preferred execution form (EXEC_PERSISTENT/PLAIN/ASYNC)."""
        _check(load().gltrsv_plan_set_exec(self._p, int(form)), "gltrsv_plan_set_exec")

    def tune(self, b=None, x=None, reps: int = 5, stream=None) -> dict:
        """Times the plan's execution forms and makes the fastest the
        preferred one; returns {"form": name, "us": {name: microseconds}}
        (the one-workgroup form only for plans built with exec_hint 2).
        b defaults to ones; b and x must not overlap."""
        import torch
        if b is None:
            b = torch.ones(self.n, dtype=torch.float64, device="cuda")
        if x is None:
            x = torch.empty_like(b)
        us = (ctypes.c_double * EXEC_FORMS)()
        best = i32(0)
        _check(load().gltrsv_plan_tune(self._p, _dev_ptr(b, self.n), _dev_ptr(x, self.n), int(reps),
                                       _stream_ptr(stream), us, ctypes.byref(best)), "gltrsv_plan_tune")
        return {"form": EXEC_NAMES[best.value],
                "us": {EXEC_NAMES[f]: us[f] for f in range(EXEC_FORMS) if us[f] >= 0.0}}

    def set_steal_wait(self, microseconds: int):
        """Superstep wait after which the persistent solve robs workgroups
        that have not started (0 = at the first wait)."""
        _check(load().gltrsv_plan_set_steal_wait(self._p, int(microseconds)), "gltrsv_plan_set_steal_wait")

    def set_start_delay(self, microseconds: int):
        """Diagnostic: every 7th workgroup of the persistent solve starts this
        much later (exercises the robbing of workgroups that have not
        started)."""
        _check(load().gltrsv_plan_set_start_delay(self._p, int(microseconds)), "gltrsv_plan_set_start_delay")

    def set_spin_limit(self, polls: int):
        """Polls a device-side wait may take before the solve reports a time-out."""
        _check(load().gltrsv_plan_set_spin_limit(self._p, int(polls)), "gltrsv_plan_set_spin_limit")

    def solve_async(self, b, x=None, stream=None):
        """Semi-asynchronous solve: no barriers, per-row readiness."""
        import torch
        if x is None:
            x = torch.empty_like(b)
        _check(load().gltrsv_solve_async(self._p, _dev_ptr(b, self.n), _dev_ptr(x, self.n), _stream_ptr(stream)),
               "gltrsv_solve_async")
        return x

    def solve_local(self, b, x=None, stream=None):
        """One-workgroup solve (plans built with exec_hint=2)."""
        import torch
        if x is None:
            x = torch.empty_like(b)
        _check(load().gltrsv_solve_local(self._p, _dev_ptr(b, self.n), _dev_ptr(x, self.n), _stream_ptr(stream)),
               "gltrsv_solve_local")
        return x

    def local_records(self):
        """The one-workgroup layout: (records as uint8, info as uint32 [records, 4])."""
        nb, nr = i64(0), i64(0)
        _check(load().gltrsv_plan_local_size(self._p, ctypes.byref(nb), ctypes.byref(nr)), "gltrsv_plan_local_size")
        rec = np.empty(max(1, nb.value), dtype=np.uint8)
        info = np.empty((max(1, nr.value), 4), dtype=np.uint32)
        _check(load().gltrsv_plan_local_records(self._p, _np_ptr(rec), nb.value, _np_ptr(info), nr.value),
               "gltrsv_plan_local_records")
        return rec[:nb.value], info[:nr.value]

    def solve_multi(self, b, x=None, stream=None):
        """Several right-hand sides: b and x are (n, nrhs) row-major CUDA
        float64 tensors; column r of x solves column r of b."""
        import torch
        if not isinstance(b, torch.Tensor) or b.dim() != 2 or b.shape[0] != self.n:
            raise ValueError("b must be an (n, nrhs) tensor")
        if x is None:
            x = torch.empty_like(b)
        if not isinstance(x, torch.Tensor) or x.shape != b.shape:
            raise ValueError("x must have b's shape")
        nrhs = int(b.shape[1])
        bp = _dev_ptr(b, self.n * nrhs)
        xp = _dev_ptr(x, self.n * nrhs)
        _check(load().gltrsv_solve_multi(self._p, bp, xp, nrhs, _stream_ptr(stream)), "gltrsv_solve_multi")
        return x

    def solve_plain(self, b, x=None, stream=None):
        """One kernel launch per superstep."""
        import torch
        if x is None:
            x = torch.empty_like(b)
        _check(load().gltrsv_solve_plain(self._p, _dev_ptr(b, self.n), _dev_ptr(x, self.n), _stream_ptr(stream)),
               "gltrsv_solve_plain")
        return x

    def stream(self):
        """The packed stream as (word uint32[slots], value float64[slots])."""
        slots = self.info()["stream_slots"]
        w = np.empty(slots, dtype=np.uint32)
        v = np.empty(slots, dtype=np.float64)
        _check(load().gltrsv_plan_stream(self._p, _np_ptr(w), _np_ptr(v), slots), "gltrsv_plan_stream")
        return w, v

    def gather_probe(self, x, y=None, stream=None):
        """The solve's traffic without its dependencies (diagnostic):
        y[i] = running sum of A_ij * x_j over row i's off-diagonals, 1.0 in
        place of x_j for the entries the solve keeps on chip."""
        import torch
        if y is None:
            y = torch.zeros_like(x)
        _check(load().gltrsv_plan_gather_probe(self._p, _dev_ptr(x, self.n), _dev_ptr(y, self.n), _stream_ptr(stream)),
               "gltrsv_plan_gather_probe")
        return y

    def debug_trace(self):
        """[S, grid, 3] wall-clock stamps of the last persistent solve (trace
        builds only)."""
        inf = self.info()
        S, G = inf["supersteps"], inf["grid_blocks"]
        out = np.zeros(S * G * 3, dtype=np.int64)
        _check(load().gltrsv_debug_trace(self._p, _np_ptr(out), out.size), "gltrsv_debug_trace")
        return out.reshape(S, G, 3)

    def device_status(self) -> int:
        st = ctypes.c_int32(0)
        _check(load().gltrsv_plan_device_status(self._p, ctypes.byref(st)), "gltrsv_plan_device_status")
        return st.value


def _ptr_array(tensors, n_of):
    arr = (ctypes.c_void_p * len(tensors))()
    for i, t in enumerate(tensors):
        arr[i] = _dev_ptr(t, n_of(i)).value
    return arr


class Batch:
    """Several plans solved together in one persistent launch."""

    def __init__(self, plans, per_claim: int = 1, use_graph: bool = True, grid_blocks: int = 0,
                 async_exec: bool = False):
        self.plans = list(plans)
        o = BatchOpts()
        load().gltrsv_default_batch_opts(ctypes.byref(o))
        o.per_claim, o.use_graph, o.grid_blocks = int(per_claim), int(bool(use_graph)), int(grid_blocks)
        o.async_exec = int(bool(async_exec))
        handles = (ctypes.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        ptr = ctypes.c_void_p()
        _check(load().gltrsv_batch_create(handles, len(self.plans), ctypes.byref(o), ctypes.byref(ptr)),
               "gltrsv_batch_create")
        self._p = ptr

    def close(self):
        if self._p:
            load().gltrsv_batch_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def info(self):
        s, g = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(load().gltrsv_batch_info(self._p, ctypes.byref(s), ctypes.byref(g)), "gltrsv_batch_info")
        return {"systems": s.value, "grid_blocks": g.value}

    def solve(self, bs, xs, stream=None):
        bp = _ptr_array(bs, lambda i: self.plans[i].n)
        xp = _ptr_array(xs, lambda i: self.plans[i].n)
        _check(load().gltrsv_batch_solve(self._p, bp, xp, _stream_ptr(stream)), "gltrsv_batch_solve")
        return xs

    def status(self) -> int:
        st = ctypes.c_int32(0)
        _check(load().gltrsv_batch_status(self._p, ctypes.byref(st)), "gltrsv_batch_status")
        return st.value


def solve_batched(plans, bs, xs, stream=None):
    """One-shot batched solve (synchronises the stream)."""
    handles = (ctypes.c_void_p * len(plans))(*[p.handle.value for p in plans])
    bp = _ptr_array(bs, lambda i: plans[i].n)
    xp = _ptr_array(xs, lambda i: plans[i].n)
    _check(load().gltrsv_solve_batched(handles, bp, xp, len(plans), _stream_ptr(stream)), "gltrsv_solve_batched")
    return xs


def solve_batched_noalloc(plans, bs, xs, stream=None):
    """As solve_batched, with the batch state in the library's fixed device
    array instead of per-call allocations (synchronises the stream)."""
    handles = (ctypes.c_void_p * len(plans))(*[p.handle.value for p in plans])
    bp = _ptr_array(bs, lambda i: plans[i].n)
    xp = _ptr_array(xs, lambda i: plans[i].n)
    _check(load().gltrsv_solve_batched_noalloc(handles, bp, xp, len(plans), _stream_ptr(stream)),
           "gltrsv_solve_batched_noalloc")
    return xs


GLTRSV_EAGAIN = -7


def clock_ns() -> int:
    return int(load().gltrsv_clock_ns())


class Server:
    """Continuous-batching solve server (worker thread inside the library)."""

    def __init__(self, **overrides):
        o = ServerOpts()
        load().gltrsv_default_server_opts(ctypes.byref(o))
        for k, v in overrides.items():
            if not hasattr(o, k):
                raise KeyError(k)
            setattr(o, k, v)
        self.opts = o
        ptr = ctypes.c_void_p()
        _check(load().gltrsv_server_create(ctypes.byref(o), ctypes.byref(ptr)), "gltrsv_server_create")
        self._p = ptr
        # ticket -> (plan, b, x): the device may use them until the ticket is
        # polled or cancelled, so the binding keeps them alive until then
        self._held = {}

    def submit(self, plan, b, x):
        """Returns a ticket, or None when the in-flight budget is full (EAGAIN)."""
        t = ctypes.c_uint64(0)
        rc = load().gltrsv_server_submit(self._p, plan.handle, _dev_ptr(b, plan.n), _dev_ptr(x, plan.n),
                                         ctypes.byref(t))
        if rc == GLTRSV_EAGAIN:
            return None
        _check(rc, "gltrsv_server_submit")
        self._held[t.value] = (plan, b, x)
        return t.value

    def poll(self, max_items: int = 4096):
        tk = (ctypes.c_uint64 * max_items)()
        ns = (ctypes.c_int64 * max_items)()
        k = ctypes.c_int32(0)
        _check(load().gltrsv_server_poll(self._p, tk, ns, max_items, ctypes.byref(k)), "gltrsv_server_poll")
        out = [(tk[i], ns[i]) for i in range(k.value)]
        for t, _ in out:
            self._held.pop(t, None)
        return out

    def cancel(self, ticket: int) -> bool:
        """Withdraws a pending request (never reported by poll afterwards);
        returns once the device no longer uses its b, x and plan.  False if
        no pending request has this ticket."""
        rc = load().gltrsv_server_cancel(self._p, ctypes.c_uint64(int(ticket)))
        if rc == -11:
            return False
        _check(rc, "gltrsv_server_cancel")
        self._held.pop(int(ticket), None)
        return True

    def stats(self) -> dict:
        st = ServerStats()
        _check(load().gltrsv_server_get_stats(self._p, ctypes.byref(st)), "gltrsv_server_get_stats")
        return st.as_dict()

    def close(self):
        if self._p:
            load().gltrsv_server_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
