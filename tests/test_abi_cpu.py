"""Host-side checks of libfwi.so that need no GPU.

The library loads, exports every entry point include/fwi.h declares, and its
host-only logic is right: argument validation happens before any device
call, workspace sizing, the stability limit, and the revolve checkpointing
schedule (optimal step count against a brute-force dynamic programme and the
closed-form binomial bound; validity by replaying it on a fake executor).
"""
import ctypes
import functools
import math
import os
import re

import pytest

import oracle
from paper_1912_08063_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _prob(**kw):
    p = _lib.FwiProblem()
    p.ndim = kw.get("ndim", 2)
    for i, n in enumerate(kw.get("shape", (64, 80))):
        p.shape[i] = n
    p.dx = kw.get("dx", 10.0)
    p.dt = kw.get("dt", 1e-3)
    p.nt = kw.get("nt", 100)
    p.order = kw.get("order", 8)
    p.nsponge = kw.get("nsponge", 10)
    p.eta_max = kw.get("eta_max", 100.0)
    p.nshots = kw.get("nshots", 1)
    p.nrec = kw.get("nrec", 5)
    return p


def test_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "fwi.h")).read()
    declared = set(re.findall(r"^(?:int|void|const char \*)\s*(fwi_\w+)\(", header, re.M))
    assert declared == set(_lib.EXPORTS)
    lib = _lib.load()
    for name in declared:
        assert hasattr(lib, name), name


def test_strerror_and_last_error():
    lib = _lib.load()
    assert lib.fwi_strerror(0) == b"ok"
    assert b"stability" in lib.fwi_strerror(_lib.FWI_ECFL)
    assert lib.fwi_strerror(12345) == b"unknown status"


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("order", [2, 4, 8, 16])
def test_cfl_limit_matches_oracle(ndim, order):
    assert abs(_lib.fwi_cfl_limit(ndim, order) - oracle.cfl_limit(ndim, order)) < 1e-6


@pytest.mark.parametrize("bad", [dict(ndim=4), dict(order=6), dict(dx=0.0), dict(dt=-1.0),
                                 dict(nt=0), dict(nsponge=-1), dict(eta_max=float("nan")),
                                 dict(nshots=0), dict(nrec=-2), dict(shape=(0, 10))])
def test_invalid_problems_rejected_before_any_device_call(bad):
    p = _prob(**bad)
    with pytest.raises(_lib.FwiError) as e:
        _lib.fwi_workspace_bytes(p, _lib.MODE_FORWARD)
    assert e.value.status == _lib.FWI_EINVAL
    lib = _lib.load()
    # the entry points validate the problem before touching any pointer
    st = lib.fwi_forward(ctypes.byref(p), None, None, None, None, None, None, 0, None)
    assert st == _lib.FWI_EINVAL


def test_tile_probe_rejects_bad_arguments_before_any_device_call():
    lib = _lib.load()
    a, b, c, o = (ctypes.c_void_p(x) for x in (0x1000, 0x2000, 0x3000, 0x4000))
    zc = ctypes.c_int32(-1)
    bad = [
        (None, b, c, o, 8, 8, 8, 0, 0),      # NULL field
        (a, b, c, a, 8, 8, 8, 0, 0),         # out equal to an input
        (a, b, c, o, 0, 8, 8, 0, 0),         # empty grid
        (a, b, c, o, 8, 8, 1 << 21, 0, 0),   # dimension out of range
        (a, b, c, o, 8, 1 << 20, 1 << 20, 0, 0),  # plane of 2^31 bytes or more
        (a, b, c, o, 8, 8, 8, -1, 0),        # negative chunk length
        (a, b, c, o, 8, 8, 8, 0, 10),        # unknown mode
    ]
    for args in bad:
        assert lib.fwi_tile_probe(*args, ctypes.byref(zc), None) == _lib.FWI_EINVAL, args
    assert zc.value == -1


def test_workspace_too_small_is_enomem_without_device():
    p = _prob()
    lib = _lib.load()
    need = _lib.fwi_workspace_bytes(p, _lib.MODE_FORWARD)
    st = lib.fwi_forward(ctypes.byref(p), None, None, None, None, None, 256, need - 1, None)
    assert st == _lib.FWI_ENOMEM


def test_workspace_sizes_grow_with_the_policy():
    p = _prob(nt=300, nshots=4)
    f = _lib.fwi_workspace_bytes(p, _lib.MODE_FORWARD)
    ck_all = _lib.FwiCkpt(kind=_lib.CKPT_ALL)
    ck_e = _lib.FwiCkpt(kind=_lib.CKPT_EVERY, every=30)
    ck_r = _lib.FwiCkpt(kind=_lib.CKPT_REVOLVE, slots=5)
    g_all = _lib.fwi_workspace_bytes(p, _lib.MODE_GRADIENT, ck_all)
    g_e = _lib.fwi_workspace_bytes(p, _lib.MODE_GRADIENT, ck_e)
    g_r = _lib.fwi_workspace_bytes(p, _lib.MODE_GRADIENT, ck_r)
    assert f < g_r < g_e < g_all
    # a field is at least the padded grid with its frame
    cells = (64 + 20 + 8) * (80 + 20 + 8)
    assert _lib.fwi_workspace_bytes(p, _lib.MODE_CKPT_BUF, ck_all) >= 301 * 4 * 4 * cells


def test_job_sizes_follow_the_checkpoint_policy():
    """A served gradient job is sized by its own policy: NULL means every
    `chunk` steps, as an explicit every:chunk does; a revolve job with a few
    slots needs less memory than one with a snapshot every chunk."""
    p = _prob(nt=600, nshots=1)
    every = _lib.fwi_job_bytes(p, _lib.JOB_GRADIENT, 20)
    assert every == _lib.fwi_job_bytes(p, _lib.JOB_GRADIENT, 20,
                                       _lib.FwiCkpt(kind=_lib.CKPT_EVERY, every=20))
    rev = _lib.fwi_job_bytes(p, _lib.JOB_GRADIENT, 20, _lib.FwiCkpt(kind=_lib.CKPT_REVOLVE,
                                                                    slots=4))
    assert _lib.fwi_job_bytes(p, _lib.JOB_FORWARD, 20) < rev < every
    with pytest.raises(_lib.FwiError) as e:
        _lib.fwi_job_bytes(p, _lib.JOB_GRADIENT, 20, _lib.FwiCkpt(kind=7))
    assert e.value.status == _lib.FWI_EINVAL


def test_advance_workspace_grows_with_jobs_and_steps():
    a = _lib.fwi_jobs_ws_bytes(8, 10)
    assert _lib.fwi_jobs_ws_bytes(8, 50) > a and _lib.fwi_jobs_ws_bytes(16, 10) > a
    lib = _lib.load()
    out = ctypes.c_uint64()
    assert lib.fwi_jobs_ws_bytes(8, 0, ctypes.byref(out)) == _lib.FWI_EINVAL
    assert lib.fwi_jobs_ws_bytes(-1, 4, ctypes.byref(out)) == _lib.FWI_EINVAL
    # too small a workspace is refused before any job is touched
    assert lib.fwi_jobs_advance(None, 0, 4, None, 0, None) == _lib.FWI_ENOMEM


# ------------------------------------------------------ revolve placement
def _replay_plan(nt, slots):
    """Replays the library's binomial-checkpointing launches with labelled
    fields: every field holds the time level it was last given.  Checks that
    each forward step reads levels n and n-1 and each adjoint step level k,
    that snapshot copies read the level they name, that no copy reads a field
    the same launch overwrites, and that the adjoint visits nt .. 1 once
    each."""
    plan = _lib.fwi_revolve_plan(nt, slots)
    ring = {0: 0, 1: -1}              # ring entry -> level (0 and -1: zero states)
    snap = {}                          # snapshot field -> level
    adj, fwd = [], 0
    zero = lambda L: L <= 0

    def get(L, lm):
        return snap.get(lm[L]) if L in lm else ring.get(L % 2)

    def same(have, L):
        return have == L or (zero(L) and have is not None and zero(have))

    for kind, a, b, c, lm in plan:
        if kind == 1:
            fwd += 1
            for L in (a, a - 1):
                assert same(get(L, lm), L), (nt, slots, "step", a, L, get(L, lm))
            if a + 1 in lm:
                snap[lm[a + 1]] = a + 1
            else:
                ring[(a + 1) % 2] = a + 1
        elif kind == 2:
            assert same(get(a, lm), a), (nt, slots, "adjoint", a, get(a, lm))
            adj.append(a)
        else:
            d, mask = c & 3, c >> 2
            ws = [w for w in (0, 1) if mask >> w & 1]
            if d == 0:
                dst = {2 * a + w for w in ws}
                vals = {}
                for w in ws:
                    L = b - w
                    assert not (L in lm and lm[L] in dst and lm[L] != 2 * a + w), (nt, slots, "race")
                    assert same(get(L, lm), L), (nt, slots, "snapshot source", L)
                    vals[w] = get(L, lm)
                for w in ws:
                    snap[2 * a + w] = vals[w]
            elif d == 1:
                for w in ws:
                    ring[(b - w) % 2] = snap[2 * a + w]
            else:
                ring[0], ring[1] = 0, -1
    assert adj == list(range(nt, 0, -1)), (nt, slots)
    return fwd


@pytest.mark.parametrize("slots", [0, 1, 2, 3, 5, 9, 48])
def test_revolve_placement_replays(slots):
    """The copy-free placement of levels in snapshot slots (restores read the
    slot; the steps producing a snapshot write into it), replayed from the
    library's own launch plan."""
    for nt in list(range(1, 90)) + [250, 601]:
        if slots > nt:
            continue
        fwd = _replay_plan(nt, slots)
        assert fwd == _lib.fwi_revolve_schedule(nt, min(slots, nt), with_actions=False)[1], nt


def test_revolve_placement_copies_only_where_needed():
    """Under the salt workload's schedule (3000 steps, 48 slots): no restore
    copies, no two-field snapshot copies; the only copies are the older level
    of the 2465 snapshots taken one step after the previous one, plus the
    two restarts' zero fills.  7675 forward and 3000 adjoint launches."""
    from collections import Counter
    plan = _lib.fwi_revolve_plan(3000, 48)
    kinds = Counter(p[0] for p in plan)
    assert kinds[1] == 7675 and kinds[2] == 3000
    copies = Counter((c & 3, c >> 2) for kind, a, b, c, lm in plan if kind == 3)
    assert copies == Counter({(0, 2): 2465, (2, 3): 2})


# ------------------------------------------------------------------ revolve
@functools.lru_cache(maxsize=None)
def _dp(l, s):
    """Brute force: minimal forward steps to visit states l-1..0 in reverse,
    state 0 held in one of s snapshots."""
    if l <= 1:
        return 0
    if s <= 1:
        return l * (l - 1) // 2
    return min(m + _dp(l - m, s - 1) + _dp(m, s) for m in range(1, l))


def _closed_form(l, s):
    beta = lambda s_, r_: math.comb(s_ + r_, s_) if r_ >= 0 else 0
    r = 0
    while beta(s, r) < l:
        r += 1
    return r * l - beta(s + 1, r - 1)


def test_revolve_closed_form_matches_brute_force():
    for l in range(1, 61):
        for s in range(1, 7):
            assert _dp(l, s) == _closed_form(l, s), (l, s)


def _replay(nsteps, slots, acts):
    """Fake executor: replays a schedule and checks that every adjoint visit
    sees the right forward state, in the order nsteps-1 .. 1."""
    cur = 0
    held = {}
    visits = []
    steps = 0
    started = False
    for op, arg in acts:
        if op == _lib.OP_ADVANCE:
            assert arg > cur
            steps += arg - cur
            cur = arg
        elif op == _lib.OP_TAKESHOT:
            assert 0 <= arg < slots
            held[arg] = cur
        elif op == _lib.OP_RESTORE:
            assert arg in held
            cur = held[arg]
        elif op == _lib.OP_RESTART:
            cur = 0
        elif op == _lib.OP_ADJOINT:
            assert arg == cur
            visits.append(arg)
            started = True
        else:
            raise AssertionError(op)
    assert visits == list(range(nsteps - 1, 0, -1))
    return steps


@pytest.mark.parametrize("nsteps,slots", [(1, 0), (2, 0), (7, 0), (10, 1), (10, 3), (37, 2),
                                          (60, 4), (100, 7), (200, 10), (64, 70)])
def test_revolve_schedule_is_valid_and_optimal(nsteps, slots):
    acts, fwd = _lib.fwi_revolve_schedule(nsteps, slots)
    steps = _replay(nsteps, slots, acts)
    assert fwd == steps + 1   # plus the recording sweep's last step
    # slots physical snapshots plus the free zero state
    assert steps == _dp(nsteps, slots + 1) == _closed_form(nsteps, slots + 1)


def test_revolve_large_schedule_matches_bound():
    # a 3000-step reversal with 52 snapshots (state 0 stored) costs 7515 steps;
    # with the zero state free the same 52 slots act as 53 snapshots
    assert _closed_form(3000, 52) == 7515
    _, fwd = _lib.fwi_revolve_schedule(3000, 51, with_actions=False)
    assert fwd - 1 == 7515
    acts, fwd = _lib.fwi_revolve_schedule(3000, 52)
    assert _replay(3000, 52, acts) == fwd - 1 == _closed_form(3000, 53)
