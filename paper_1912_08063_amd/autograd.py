"""FWIForward: a torch.autograd.Function whose backward is the adjoint solver.

forward():  fwi_forward_ckpt -- propagates every shot, returns the traces and
            keeps, instead of every time level, only what the checkpoint
            policy needs (every-k snapshots and a segment ring, or a revolve
            snapshot store) in one device buffer saved on the context.
backward(): fwi_backward -- recomputes the forward wavefield from those
            checkpoints, runs the adjoint propagation with grad_traces as its
            source and returns dv = d(loss)/d(v) (imaging condition).

With loss = ((traces - obs)**2).sum(), grad_traces = 2 (traces - obs), which is
the adjoint source of the least-squares misfit (Eq. 1), so v.grad equals the
dv of fwi_gradient for the same inputs.
"""
from __future__ import annotations

import torch

from . import _lib
from .api import Config, _require, _shots, make_problem, parse_ckpt, resolve_ckpt


class FWIForward(torch.autograd.Function):
    @staticmethod
    def forward(ctx, v, src, src_pos, rec_pos, cfg: Config):
        v = _require(v.detach(), "v", torch.float32)
        src = _require(src.detach(), "src", torch.float32)
        src_pos = _require(src_pos, "src_pos", torch.int32)
        rec_pos = _require(rec_pos, "rec_pos", torch.int32)
        src, src_pos, rec_pos = _shots(v, src, src_pos, rec_pos)
        S, R, nt = src_pos.shape[0], rec_pos.shape[1], src.shape[1]
        prob = make_problem(v, nt, cfg, S, R)
        ck = parse_ckpt(resolve_ckpt(cfg.ckpt, prob, v.device, "autograd"))
        stream = torch.cuda.current_stream(v.device).cuda_stream
        ck_bytes = _lib.fwi_workspace_bytes(prob, _lib.MODE_CKPT_BUF, ck)
        ws_bytes = _lib.fwi_workspace_bytes(prob, _lib.MODE_FORWARD_CKPT, ck)
        ckpt_buf = torch.empty(max(ck_bytes, 256), dtype=torch.uint8, device=v.device)
        ws = torch.empty(max(ws_bytes, 256), dtype=torch.uint8, device=v.device)
        traces = torch.empty((S, nt, R), dtype=torch.float32, device=v.device)
        _lib.fwi_forward_ckpt(prob, v.data_ptr(), src.data_ptr(), src_pos.data_ptr(),
                              rec_pos.data_ptr() if R else None,
                              ck, traces.data_ptr() if R else None, ckpt_buf.data_ptr(),
                              ckpt_buf.numel(), ws.data_ptr(), ws.numel(), stream)
        ctx.save_for_backward(v, src, src_pos, rec_pos)
        ctx.prob, ctx.ck, ctx.ckpt_buf = prob, ck, ckpt_buf
        ctx.ws_keep = ws   # keeps the job tables alive until the stream is done
        return traces

    @staticmethod
    def backward(ctx, grad_traces):
        if ctx.ckpt_buf is None:
            raise RuntimeError("FWIForward: the checkpoints were consumed by a previous "
                               "backward; run the forward again")
        v, src, src_pos, rec_pos = ctx.saved_tensors
        grad_traces = grad_traces.to(torch.float32).contiguous()
        prob, ck = ctx.prob, ctx.ck
        stream = torch.cuda.current_stream(v.device).cuda_stream
        ws_bytes = _lib.fwi_workspace_bytes(prob, _lib.MODE_BACKWARD, ck)
        ws = torch.empty(max(ws_bytes, 256), dtype=torch.uint8, device=v.device)
        dv = torch.empty_like(v)
        R = rec_pos.shape[1]
        _lib.fwi_backward(prob, v.data_ptr(), src.data_ptr(), src_pos.data_ptr(),
                          rec_pos.data_ptr() if R else None, ck, ctx.ckpt_buf.data_ptr(),
                          ctx.ckpt_buf.numel(), grad_traces.data_ptr() if R else None,
                          dv.data_ptr(), ws.data_ptr(), ws.numel(), stream)
        # the buffers must outlive the queued kernels: hand them to the stream
        ctx.ckpt_buf.record_stream(torch.cuda.current_stream(v.device))
        ws.record_stream(torch.cuda.current_stream(v.device))
        ctx.ckpt_buf = None
        return dv, None, None, None, None


def fwi_forward_op(v, src, src_pos, rec_pos, cfg: Config):
    """traces = FWIForward.apply(...), differentiable with respect to v."""
    return FWIForward.apply(v, src, src_pos, rec_pos, cfg)
