"""ctypes binding of libfwi.so: the C ABI of include/fwi.h, same entry-point names.

Argument marshalling only: every function forwards plain pointers and sizes to
the library and raises FwiError on a non-zero status.  There is no fallback:
if libfwi.so is missing or fails to load, load() raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# FWI_LIBRARY names another build of the same library (e.g. the host code
# built with sanitizers for the CPU tests); the default is the in-tree build.
LIB_PATH = os.environ.get("FWI_LIBRARY") or os.path.join(_HERE, "libfwi.so")

FWI_OK, FWI_EINVAL, FWI_ECFL, FWI_EBOUNDS, FWI_ENOMEM, FWI_EHIP, FWI_ENONFINITE, \
    FWI_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
MODE_FORWARD, MODE_GRADIENT, MODE_FORWARD_CKPT, MODE_BACKWARD, MODE_CKPT_BUF = range(5)
CKPT_ALL, CKPT_EVERY, CKPT_REVOLVE = 0, 1, 2
OP_ADVANCE, OP_TAKESHOT, OP_RESTORE, OP_ADJOINT, OP_RESTART = 1, 2, 3, 4, 5

EXPORTS = ["fwi_strerror", "fwi_last_error", "fwi_cfl_limit", "fwi_workspace_bytes",
           "fwi_forward", "fwi_forward_noalloc", "fwi_gradient", "fwi_forward_ckpt", "fwi_backward",
           "fwi_revolve_schedule", "fwi_revolve_plan", "fwi_velocity_range", "fwi_stream_probe",
           "fwi_tile_probe", "fwi_job_bytes", "fwi_job_create", "fwi_jobs_ws_bytes",
           "fwi_jobs_advance", "fwi_job_query", "fwi_job_misfit", "fwi_job_misfit_device",
           "fwi_job_destroy"]
JOB_FORWARD, JOB_GRADIENT = 0, 1


class FwiProblem(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("shape", ctypes.c_int32 * 3),
                ("dx", ctypes.c_float), ("dt", ctypes.c_float), ("nt", ctypes.c_int32),
                ("order", ctypes.c_int32), ("nsponge", ctypes.c_int32),
                ("eta_max", ctypes.c_float), ("nshots", ctypes.c_int32),
                ("nrec", ctypes.c_int32)]


class FwiCkpt(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("every", ctypes.c_int32), ("slots", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("budget_bytes", ctypes.c_uint64)]


class FwiError(RuntimeError):
    def __init__(self, status, func, detail):
        self.status = status
        super().__init__("%s: %s (%d): %s" % (func, _strerror(status), status, detail))


_lib = None


def load():
    """Load libfwi.so (built in-tree by paper_1912_08063_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FileNotFoundError("libfwi.so is not built (%s); run "
                                "`python -m paper_1912_08063_amd.build`" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, u64, i32, i64 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64
    prob = P(FwiProblem)
    ck = P(FwiCkpt)
    lib.fwi_strerror.argtypes = [ctypes.c_int]
    lib.fwi_strerror.restype = ctypes.c_char_p
    lib.fwi_last_error.argtypes = []
    lib.fwi_last_error.restype = ctypes.c_char_p
    lib.fwi_cfl_limit.argtypes = [i32, i32, P(ctypes.c_double)]
    lib.fwi_workspace_bytes.argtypes = [prob, i32, ck, P(u64)]
    lib.fwi_forward.argtypes = [prob, vp, vp, vp, vp, vp, vp, u64, vp]
    lib.fwi_forward_noalloc.argtypes = [prob, vp, vp, vp, vp, vp, vp]
    lib.fwi_gradient.argtypes = [prob, vp, vp, vp, vp, vp, ck, P(ctypes.c_double), vp, vp, vp,
                                 u64, vp]
    lib.fwi_forward_ckpt.argtypes = [prob, vp, vp, vp, vp, ck, vp, vp, u64, vp, u64, vp]
    lib.fwi_backward.argtypes = [prob, vp, vp, vp, vp, ck, vp, u64, vp, vp, vp, u64, vp]
    lib.fwi_revolve_schedule.argtypes = [i32, i32, P(i32), i64, P(i64), P(i64)]
    lib.fwi_revolve_plan.argtypes = [i32, i32, P(i32), i64, P(i64)]
    lib.fwi_velocity_range.argtypes = [vp, i64, P(ctypes.c_float), P(ctypes.c_float), vp, u64,
                                       vp]
    lib.fwi_stream_probe.argtypes = [vp, vp, vp, vp, i64, i32, vp]
    lib.fwi_tile_probe.argtypes = [vp, vp, vp, vp, i32, i32, i32, i32, i32, vp, vp]
    lib.fwi_job_bytes.argtypes = [prob, i32, i32, ck, P(u64)]
    lib.fwi_job_create.argtypes = [prob, i32, i32, ck, vp, vp, vp, vp, vp, vp, vp, vp, u64, vp,
                                   P(vp)]
    lib.fwi_jobs_ws_bytes.argtypes = [i32, i32, P(u64)]
    lib.fwi_jobs_advance.argtypes = [P(vp), i32, i32, vp, u64, vp]
    lib.fwi_job_query.argtypes = [vp, P(i32), P(i64)]
    lib.fwi_job_misfit.argtypes = [vp, P(ctypes.c_double), vp]
    lib.fwi_job_misfit_device.argtypes = [vp, P(vp)]
    lib.fwi_job_destroy.argtypes = [vp]
    lib.fwi_job_destroy.restype = None
    for name in EXPORTS:
        if name not in ("fwi_strerror", "fwi_last_error", "fwi_job_destroy"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _strerror(status):
    try:
        return load().fwi_strerror(status).decode()
    except Exception:   # message formatting only
        return "status"


def _check(status, func):
    if status != FWI_OK:
        raise FwiError(status, func, load().fwi_last_error().decode())
    return status


# ------------------------------------------------------------------ wrappers
def fwi_cfl_limit(ndim, order):
    out = ctypes.c_double()
    _check(load().fwi_cfl_limit(ndim, order, ctypes.byref(out)), "fwi_cfl_limit")
    return out.value


def fwi_workspace_bytes(prob, mode, ckpt=None):
    out = ctypes.c_uint64()
    _check(load().fwi_workspace_bytes(ctypes.byref(prob), mode,
                                      ctypes.byref(ckpt) if ckpt is not None else None,
                                      ctypes.byref(out)), "fwi_workspace_bytes")
    return out.value


def fwi_forward(prob, v, src, src_pos, rec_pos, traces, ws, ws_bytes, stream):
    _check(load().fwi_forward(ctypes.byref(prob), v, src, src_pos, rec_pos, traces, ws,
                              ws_bytes, stream), "fwi_forward")


def fwi_forward_noalloc(prob, v, src, src_pos, rec_pos, traces, stream):
    _check(load().fwi_forward_noalloc(ctypes.byref(prob), v, src, src_pos, rec_pos, traces,
                                      stream), "fwi_forward_noalloc")


def fwi_gradient(prob, v, src, src_pos, rec_pos, obs, ckpt, dv, traces_or_null, ws, ws_bytes,
                 stream):
    mis = ctypes.c_double()
    _check(load().fwi_gradient(ctypes.byref(prob), v, src, src_pos, rec_pos, obs,
                               ctypes.byref(ckpt), ctypes.byref(mis), dv, traces_or_null, ws,
                               ws_bytes, stream), "fwi_gradient")
    return mis.value


def fwi_forward_ckpt(prob, v, src, src_pos, rec_pos, ckpt, traces, ckpt_buf, ckpt_bytes, ws,
                     ws_bytes, stream):
    _check(load().fwi_forward_ckpt(ctypes.byref(prob), v, src, src_pos, rec_pos,
                                   ctypes.byref(ckpt), traces, ckpt_buf, ckpt_bytes, ws,
                                   ws_bytes, stream), "fwi_forward_ckpt")


def fwi_backward(prob, v, src, src_pos, rec_pos, ckpt, ckpt_buf, ckpt_bytes, grad_traces, dv,
                 ws, ws_bytes, stream):
    _check(load().fwi_backward(ctypes.byref(prob), v, src, src_pos, rec_pos,
                               ctypes.byref(ckpt), ckpt_buf, ckpt_bytes, grad_traces, dv, ws,
                               ws_bytes, stream), "fwi_backward")


def fwi_revolve_plan(nsteps, slots):
    """The launches of a binomial-checkpointing gradient (host only): a list of
    (kind, a, b, c, level_map) with level_map {level: snapshot field}."""
    lib = load()
    count = ctypes.c_int64()
    _check(lib.fwi_revolve_plan(nsteps, slots, None, 0, ctypes.byref(count)), "fwi_revolve_plan")
    buf = (ctypes.c_int32 * (10 * max(count.value, 1)))()
    _check(lib.fwi_revolve_plan(nsteps, slots, buf, count.value, ctypes.byref(count)),
           "fwi_revolve_plan")
    out = []
    for i in range(count.value):
        row = buf[10 * i:10 * i + 10]
        lm = {row[4 + 2 * e]: row[5 + 2 * e] for e in range(3) if row[4 + 2 * e] != -2 ** 31}
        out.append((row[0], row[1], row[2], row[3], lm))
    return out


def fwi_revolve_schedule(nsteps, slots, with_actions=True):
    """Returns (actions as a list of (op, arg), forward_steps)."""
    count = ctypes.c_int64()
    steps = ctypes.c_int64()
    lib = load()
    _check(lib.fwi_revolve_schedule(nsteps, slots, None, 0, ctypes.byref(count),
                                    ctypes.byref(steps)), "fwi_revolve_schedule")
    if not with_actions:
        return None, steps.value
    buf = (ctypes.c_int32 * (2 * max(count.value, 1)))()
    _check(lib.fwi_revolve_schedule(nsteps, slots, buf, count.value, ctypes.byref(count),
                                    ctypes.byref(steps)), "fwi_revolve_schedule")
    acts = [(buf[2 * i], buf[2 * i + 1]) for i in range(count.value)]
    return acts, steps.value


def fwi_velocity_range(v, n, ws, ws_bytes, stream):
    lo, hi = ctypes.c_float(), ctypes.c_float()
    _check(load().fwi_velocity_range(v, n, ctypes.byref(lo), ctypes.byref(hi), ws, ws_bytes,
                                     stream), "fwi_velocity_range")
    return lo.value, hi.value


def fwi_stream_probe(a, b, c, out, n, variant, stream):
    _check(load().fwi_stream_probe(a, b, c, out, n, variant, stream), "fwi_stream_probe")


def fwi_tile_probe(cur, prv, kap, out, nz, ny, nx, zc, mode, stream):
    """Returns the z-chunk length used."""
    h = ctypes.c_int32(0)
    _check(load().fwi_tile_probe(cur, prv, kap, out, nz, ny, nx, zc, mode, ctypes.byref(h),
                                 stream), "fwi_tile_probe")
    return h.value


def fwi_job_bytes(prob, kind, chunk, ckpt=None):
    out = ctypes.c_uint64()
    _check(load().fwi_job_bytes(ctypes.byref(prob), kind, chunk,
                                ctypes.byref(ckpt) if ckpt is not None else None,
                                ctypes.byref(out)), "fwi_job_bytes")
    return out.value


def fwi_job_create(prob, kind, chunk, ckpt, v, src, src_pos, rec_pos, obs, traces, dv, mem,
                   mem_bytes, stream):
    h = ctypes.c_void_p()
    _check(load().fwi_job_create(ctypes.byref(prob), kind, chunk,
                                 ctypes.byref(ckpt) if ckpt is not None else None, v, src,
                                 src_pos, rec_pos, obs, traces, dv, mem, mem_bytes, stream,
                                 ctypes.byref(h)), "fwi_job_create")
    return h


def fwi_jobs_ws_bytes(njobs, ksteps):
    out = ctypes.c_uint64()
    _check(load().fwi_jobs_ws_bytes(njobs, ksteps, ctypes.byref(out)), "fwi_jobs_ws_bytes")
    return out.value


def fwi_jobs_advance(handles, ksteps, ws, ws_bytes, stream):
    arr = (ctypes.c_void_p * max(len(handles), 1))(*[h.value for h in handles])
    _check(load().fwi_jobs_advance(arr, len(handles), ksteps, ws, ws_bytes, stream),
           "fwi_jobs_advance")


def fwi_job_query(handle):
    done = ctypes.c_int32()
    left = ctypes.c_int64()
    _check(load().fwi_job_query(handle, ctypes.byref(done), ctypes.byref(left)),
           "fwi_job_query")
    return bool(done.value), left.value


def fwi_job_misfit(handle, stream):
    out = ctypes.c_double()
    _check(load().fwi_job_misfit(handle, ctypes.byref(out), stream), "fwi_job_misfit")
    return out.value


def fwi_job_misfit_device(handle):
    out = ctypes.c_void_p()
    _check(load().fwi_job_misfit_device(handle, ctypes.byref(out)), "fwi_job_misfit_device")
    return out.value


def fwi_job_destroy(handle):
    load().fwi_job_destroy(handle)
