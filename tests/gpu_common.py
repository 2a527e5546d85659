"""Helpers shared by the GPU tests: run a workload through the HIP library and
through the FP64 oracle on the same (fp32-rounded) inputs."""
import dataclasses

import numpy as np

import oracle
from paper_1912_08063_amd import workloads as wl


def f32(P: wl.Problem) -> wl.Problem:
    """The same problem with every floating input rounded to fp32, so that the
    oracle sees exactly the numbers the library receives."""
    r = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    return dataclasses.replace(
        P, v=r(P.v), dx=float(np.float32(P.dx)), dt=float(np.float32(P.dt)),
        eta_max=float(np.float32(P.eta_max)), wavelet=r(P.wavelet),
        v_start=None if P.v_start is None else r(P.v_start))


def dev(a, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda").to(dtype)


def cfg(P, ckpt="all"):
    from paper_1912_08063_amd import api
    return api.Config(dt=P.dt, dx=P.dx, order=P.order, nsponge=P.nb, eta_max=P.eta_max,
                      ckpt=ckpt)


def inputs(P, v=None):
    import torch
    v = P.v if v is None else v
    return (dev(v, torch.float32), dev(P.wavelet, torch.float32),
            dev(P.src_pos, torch.int32), dev(P.rec_pos, torch.int32))


def gpu_forward(P):
    import torch
    from paper_1912_08063_amd import api
    v, w, s, r = inputs(P)
    tr = api.forward(v, w, s, r, cfg(P))
    torch.cuda.synchronize()
    return tr.cpu().numpy().astype(np.float64)


def oracle_forward(P, v=None):
    v = P.v if v is None else v
    return oracle.forward(v, P.wavelet, P.src_pos, P.rec_pos, P.dx, P.dt, P.order, P.nb,
                          P.eta_max)


def gpu_gradient(P, v, obs, ckpt="all"):
    import torch
    from paper_1912_08063_amd import api
    vt, w, s, r = inputs(P, v)
    mis, dv, tr = api.gradient(vt, dev(obs, torch.float32), w, s, r, cfg(P, ckpt),
                               return_traces=True)
    torch.cuda.synchronize()
    return mis, dv.cpu().numpy().astype(np.float64), tr.cpu().numpy().astype(np.float64)


def oracle_gradient(P, v, obs):
    return oracle.gradient(v, P.wavelet, P.src_pos, P.rec_pos, obs, P.dx, P.dt, P.order, P.nb,
                           P.eta_max)


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a)
