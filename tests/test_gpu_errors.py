"""Error paths through the C ABI on the GPU: every check happens on the host
before any kernel runs, and no output is written on error."""
import numpy as np
import pytest

from gpu_common import cfg, f32, inputs
from paper_1912_08063_amd import _lib, api
from paper_1912_08063_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _run(P, v=None, rec=None, src=None, dt=None):
    import torch
    vt, w, s, r = inputs(P, v)
    if rec is not None:
        r = torch.as_tensor(rec, dtype=torch.int32, device="cuda")
    if src is not None:
        s = torch.as_tensor(src, dtype=torch.int32, device="cuda")
    c = cfg(P)
    if dt is not None:
        c = api.Config(dt=dt, dx=c.dx, order=c.order, nsponge=c.nsponge, eta_max=c.eta_max)
    out = torch.full((P.nshots, P.nt, r.shape[-2]), 7.0, device="cuda")
    try:
        api.forward(vt, w, s, r, c, out=out)
        status = 0
    except _lib.FwiError as e:
        status = e.status
    torch.cuda.synchronize()
    return status, out


def test_receiver_out_of_bounds():
    P = f32(wl.small_2d(nz=30, nx=70, nt=20, nrec=3))
    rec = P.rec_pos.copy()
    rec[0, 1] = [30, 5]
    st, out = _run(P, rec=rec)
    assert st == _lib.FWI_EBOUNDS
    assert float(out.min()) == 7.0 and float(out.max()) == 7.0


def test_source_out_of_bounds():
    P = f32(wl.small_3d(shape=(10, 11, 12), nt=5, nrec=2))
    st, out = _run(P, src=[[0, 11, 0]])
    assert st == _lib.FWI_EBOUNDS


def test_cfl_violation():
    P = f32(wl.small_2d(nz=30, nx=70, nt=20, nrec=3))
    lim = _lib.fwi_cfl_limit(2, 8)
    st, out = _run(P, dt=1.01 * lim * P.dx / P.v.max())
    assert st == _lib.FWI_ECFL
    assert float(out.max()) == 7.0
    st, _ = _run(P, dt=0.99 * lim * P.dx / P.v.max())
    assert st == 0


def test_bad_velocity():
    P = f32(wl.small_2d(nz=30, nx=70, nt=20, nrec=3))
    v = P.v.copy()
    v[3, 4] = np.nan
    assert _run(P, v=v)[0] == _lib.FWI_EINVAL
    v = P.v.copy()
    v[3, 4] = 0.0
    assert _run(P, v=v)[0] == _lib.FWI_EINVAL


def test_workspace_too_small():
    import ctypes
    import torch
    P = f32(wl.small_2d(nz=30, nx=70, nt=20, nrec=3))
    vt, w, s, r = inputs(P)
    prob = api.make_problem(vt, P.nt, cfg(P), 1, 3)
    need = _lib.fwi_workspace_bytes(prob, _lib.MODE_FORWARD)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    out = torch.full((1, P.nt, 3), 7.0, device="cuda")
    st = _lib.load().fwi_forward(ctypes.byref(prob), vt.data_ptr(), w.data_ptr(), s.data_ptr(),
                                 r.data_ptr(), out.data_ptr(), ws.data_ptr(), need - 256, None)
    assert st == _lib.FWI_ENOMEM
    torch.cuda.synchronize()
    assert float(out.max()) == 7.0
