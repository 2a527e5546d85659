"""torch-level entry points: forward() and gradient() on device tensors.

torch supplies device memory (tensors, workspaces from its caching allocator)
and the stream; every step of the computation runs in libfwi.so's kernels.
Shapes follow include/fwi.h: v [nz][nx] or [nz][ny][nx] float32, src
[S][nt] float32, src_pos [S][D] int32, rec_pos [S][R][D] (or [R][D], shared
by every shot) int32, traces [S][nt][R] float32.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import torch

from . import _lib


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


def _require(t: torch.Tensor, name: str, dtype: torch.dtype):
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if t.device.type != "cuda":
        raise ValueError("%s must be a device (cuda) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    return t.contiguous()


@dataclasses.dataclass(frozen=True)
class Config:
    """Discretisation shared by forward/gradient calls."""
    dt: float
    dx: float
    order: int = 8
    nsponge: int = 20
    eta_max: Optional[float] = None   # None: the library's 3 vmax ln(1000) / (2 nsponge dx)
    # "all", "every:K", "revolve:SLOTS", "revolve:BUDGETe9B", or "auto" /
    # "auto:BUDGETe9B": the fastest of those that fits the device memory
    # (default budget: 90 % of the free memory) -- see choose_ckpt
    ckpt: str = "every:50"


def choose_ckpt(prob: "_lib.FwiProblem", budget_bytes: float, mode: str = "gradient") -> str:
    """The fastest checkpoint policy whose device memory fits budget_bytes, for
    a gradient (mode "gradient": its workspace) or a differentiable forward
    (mode "autograd": workspace plus checkpoint buffer).

    Keeping every level ("all") recomputes nothing.  Every-K snapshots
    recompute about one forward step per time step whatever K is, so the K
    that needs least memory is taken (near sqrt(2 nt): K + 1 ring levels
    plus 2 nt / K snapshot levels).  Binomial checkpointing within the budget
    recomputes more and comes last."""
    def need(spec):
        ck = parse_ckpt(spec)
        if mode == "autograd":
            return (_lib.fwi_workspace_bytes(prob, _lib.MODE_FORWARD_CKPT, ck) +
                    _lib.fwi_workspace_bytes(prob, _lib.MODE_CKPT_BUF, ck))
        return _lib.fwi_workspace_bytes(prob, _lib.MODE_GRADIENT, ck)

    if need("all") <= budget_bytes:
        return "all"
    nt = int(prob.nt)
    k0 = max(1, int(round(math.sqrt(2 * nt))))
    every = min(("every:%d" % k for k in range(max(1, k0 // 2), min(nt, 2 * k0) + 1)), key=need)
    if need(every) <= budget_bytes:
        return every
    # snapshot budget of the binomial schedule: what is left beside one slot's
    # fixed part
    slot = need("revolve:2") - need("revolve:1")
    base = need("revolve:1") - slot
    return "revolve:%.6e" % max(0.0, float(budget_bytes) - base)


def resolve_ckpt(spec: str, prob: "_lib.FwiProblem", device, mode: str = "gradient") -> str:
    """A checkpoint spec with "auto" resolved for this problem (see choose_ckpt)."""
    if not spec.startswith("auto"):
        return spec
    if ":" in spec:
        budget = float(spec.split(":", 1)[1])
    else:
        free, _ = torch.cuda.mem_get_info(device)
        budget = 0.9 * free
    return choose_ckpt(prob, budget, mode)


def parse_ckpt(spec: str) -> _lib.FwiCkpt:
    c = _lib.FwiCkpt()
    if spec == "all":
        c.kind = _lib.CKPT_ALL
    elif spec.startswith("every:"):
        c.kind = _lib.CKPT_EVERY
        c.every = int(spec.split(":")[1])
    elif spec.startswith("revolve:"):
        c.kind = _lib.CKPT_REVOLVE
        arg = spec.split(":")[1]
        if "e" in arg or "." in arg:   # a byte budget such as 40e9
            c.budget_bytes = int(float(arg))
        else:
            c.slots = int(arg)
    else:
        raise ValueError("checkpoint spec must be all, every:K or revolve:SLOTS|BUDGET")
    return c


def _shots(v, src, src_pos, rec_pos, nt=None):
    """Brings the inputs to the library's layout and checks every shape against
    the problem: the C ABI takes no array lengths, so an array shorter than the
    problem implies would be read or written out of bounds.

    src [S][L] or [L] (one wavelet for every shot), src_pos [S][D] or [D],
    rec_pos [S][R][D] or [R][D] (shared by every shot); nt <= L steps (default
    L).  Returns src [S][nt], src_pos [S][D], rec_pos [S][R][D], contiguous."""
    D = v.dim()
    if D not in (2, 3):
        raise ValueError("v must be 2-D or 3-D")
    for name, t in (("src", src), ("src_pos", src_pos), ("rec_pos", rec_pos)):
        if t.device != v.device:
            raise ValueError("%s is on %s, v on %s" % (name, t.device, v.device))
    if src_pos.dim() not in (1, 2) or src_pos.shape[-1] != D:
        raise ValueError("src_pos must be [S][%d] or [%d], got %s" % (D, D, tuple(src_pos.shape)))
    src_pos = src_pos.reshape(-1, D)
    S = src_pos.shape[0]
    if S < 1:
        raise ValueError("no shots")
    if src.dim() == 1:
        src = src.unsqueeze(0)
    if src.dim() != 2 or src.shape[0] not in (1, S):
        raise ValueError("src must be [S][nt] or [nt] with S = %d, got %s" % (S, tuple(src.shape)))
    nt = src.shape[1] if nt is None else int(nt)
    if not 1 <= nt <= src.shape[1]:
        raise ValueError("nt = %d needs 1 <= nt <= %d (the wavelet length)" % (nt, src.shape[1]))
    src = src[:, :nt].expand(S, nt)
    if rec_pos.dim() == 2 and rec_pos.shape[-1] == D:
        rec_pos = rec_pos.unsqueeze(0).expand(S, rec_pos.shape[0], D)
    if rec_pos.dim() != 3 or rec_pos.shape[0] != S or rec_pos.shape[2] != D:
        raise ValueError("rec_pos must be [%d][R][%d] or [R][%d], got %s"
                         % (S, D, D, tuple(rec_pos.shape)))
    return src.contiguous(), src_pos.contiguous(), rec_pos.contiguous()


def _check_traces(t, name, S, nt, R, device):
    """obs / out arrays: [S][nt][R] float32 on the model's device."""
    if tuple(t.shape) != (S, nt, R):
        raise ValueError("%s must be [%d][%d][%d], got %s" % (name, S, nt, R, tuple(t.shape)))
    if t.device != device:
        raise ValueError("%s is on %s, v on %s" % (name, t.device, device))


def default_eta_max(vmax: float, nsponge: int, dx: float) -> float:
    if nsponge <= 0:
        return 0.0
    return 3.0 * vmax * math.log(1000.0) / (2.0 * nsponge * dx)


def velocity_range(v: torch.Tensor):
    v = _require(v, "v", torch.float32)
    ws = torch.empty(4096, dtype=torch.uint8, device=v.device)
    return _lib.fwi_velocity_range(v.data_ptr(), v.numel(), ws.data_ptr(), ws.numel(),
                                   torch.cuda.current_stream(v.device).cuda_stream)


def make_problem(v, nt, cfg: Config, nshots, nrec) -> _lib.FwiProblem:
    p = _lib.FwiProblem()
    p.ndim = v.dim()
    for i, n in enumerate(v.shape):
        p.shape[i] = int(n)
    p.dx, p.dt, p.nt = float(cfg.dx), float(cfg.dt), int(nt)
    p.order, p.nsponge = int(cfg.order), int(cfg.nsponge)
    # a negative eta_max asks the library for its default from the model's v_max
    p.eta_max = -1.0 if cfg.eta_max is None else float(cfg.eta_max)
    p.nshots, p.nrec = int(nshots), int(nrec)
    return p


class Workspace:
    """A reusable device workspace (grows on demand, 256-byte aligned via torch)."""

    def __init__(self, device=None):
        self.device = device
        self.buf = None

    def get(self, nbytes, device):
        nbytes = max(int(nbytes), 256)
        if self.buf is None or self.buf.numel() < nbytes or self.buf.device != device:
            self.buf = None
            self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        return self.buf


def forward(v, src, src_pos, rec_pos, cfg: Config, nt: Optional[int] = None,
            workspace: Optional[Workspace] = None, out: Optional[torch.Tensor] = None):
    """Forward modelling through fwi_forward; returns traces [S][nt][R]."""
    v = _require(v, "v", torch.float32)
    src = _require(src, "src", torch.float32)
    src_pos = _require(src_pos, "src_pos", torch.int32)
    rec_pos = _require(rec_pos, "rec_pos", torch.int32)
    src, src_pos, rec_pos = _shots(v, src, src_pos, rec_pos, nt)
    S, R, nt = src_pos.shape[0], rec_pos.shape[1], src.shape[1]
    prob = make_problem(v, nt, cfg, S, R)
    nbytes = _lib.fwi_workspace_bytes(prob, _lib.MODE_FORWARD)
    ws = (workspace or Workspace()).get(nbytes, v.device)
    if out is not None:
        _check_traces(out, "out", S, nt, R, v.device)
        if out.dtype != torch.float32 or not out.is_contiguous():
            raise ValueError("out must be a contiguous float32 tensor")
    traces = out if out is not None else torch.empty((S, nt, R), dtype=torch.float32,
                                                     device=v.device)
    _lib.fwi_forward(prob, v.data_ptr(), src.data_ptr(), src_pos.data_ptr(),
                     _ptr(rec_pos) if R else None, _ptr(traces) if R else None,
                     ws.data_ptr(), ws.numel(), torch.cuda.current_stream(v.device).cuda_stream)
    return traces


def gradient(v, obs, src, src_pos, rec_pos, cfg: Config, return_traces=False,
             workspace: Optional[Workspace] = None):
    """Misfit (Eq. 1) and d(misfit)/d(v) through fwi_gradient."""
    v = _require(v, "v", torch.float32)
    obs = _require(obs, "obs", torch.float32)
    src = _require(src, "src", torch.float32)
    src_pos = _require(src_pos, "src_pos", torch.int32)
    rec_pos = _require(rec_pos, "rec_pos", torch.int32)
    src, src_pos, rec_pos = _shots(v, src, src_pos, rec_pos)
    S, R, nt = src_pos.shape[0], rec_pos.shape[1], src.shape[1]
    _check_traces(obs, "obs", S, nt, R, v.device)
    prob = make_problem(v, nt, cfg, S, R)
    ck = parse_ckpt(resolve_ckpt(cfg.ckpt, prob, v.device))
    nbytes = _lib.fwi_workspace_bytes(prob, _lib.MODE_GRADIENT, ck)
    ws = (workspace or Workspace()).get(nbytes, v.device)
    dv = torch.empty_like(v)
    traces = torch.empty((S, nt, R), dtype=torch.float32, device=v.device) if return_traces else None
    mis = _lib.fwi_gradient(prob, v.data_ptr(), src.data_ptr(), src_pos.data_ptr(),
                            _ptr(rec_pos) if R else None, _ptr(obs) if R else None, ck,
                            dv.data_ptr(), _ptr(traces), ws.data_ptr(), ws.numel(),
                            torch.cuda.current_stream(v.device).cuda_stream)
    if return_traces:
        return mis, dv, traces
    return mis, dv
