"""Shape checks of the torch binding (CPU tensors; no GPU needed).

The C ABI takes no array lengths -- every length follows from the problem --
so the binding must refuse any array shorter or shaped differently than the
problem implies before it passes a pointer on."""
import pytest
import torch

from paper_1912_08063_amd.api import _check_traces, _shots

I32, F32 = torch.int32, torch.float32


def _ins(D=2, S=3, R=5, L=40):
    v = torch.ones((8,) * D, dtype=F32)
    return (v, torch.zeros(S, L, dtype=F32), torch.zeros(S, D, dtype=I32),
            torch.zeros(S, R, D, dtype=I32))


@pytest.mark.parametrize("D", [2, 3])
def test_layouts_accepted(D):
    v, src, sp, rp = _ins(D)
    s, p, r = _shots(v, src, sp, rp)
    assert s.shape == (3, 40) and p.shape == (3, D) and r.shape == (3, 5, D)
    # one wavelet and one receiver line shared by every shot
    s, p, r = _shots(v, src[0], sp, rp[0])
    assert s.shape == (3, 40) and r.shape == (3, 5, D) and s.is_contiguous()
    # a single shot given as flat positions
    s, p, r = _shots(v, src[:1], sp[0], rp[0])
    assert s.shape == (1, 40) and p.shape == (1, D) and r.shape == (1, 5, D)
    # fewer steps than the wavelet: each shot's row is cut, not re-strided
    src2 = torch.arange(3 * 40, dtype=F32).reshape(3, 40)
    s, _, _ = _shots(v, src2, sp, rp, nt=7)
    assert s.shape == (3, 7) and s.is_contiguous() and float(s[1, 0]) == 40.0
    # no receivers
    s, p, r = _shots(v, src, sp, rp[:, :0])
    assert r.shape == (3, 0, D)


def test_mismatches_refused():
    v, src, sp, rp = _ins()
    with pytest.raises(ValueError):
        _shots(v, src, sp, rp, nt=41)                  # longer than the wavelet
    with pytest.raises(ValueError):
        _shots(v, src, sp, rp, nt=0)
    with pytest.raises(ValueError):
        _shots(v, src[:2], sp, rp)                     # 2 wavelets for 3 shots
    with pytest.raises(ValueError):
        _shots(v, src, sp, rp[:2])                     # receivers of 2 shots
    with pytest.raises(ValueError):
        _shots(v, src, sp[:, :1], rp)                  # positions of the wrong rank
    with pytest.raises(ValueError):
        _shots(v, src, sp, torch.zeros(3, 5, 3, dtype=I32))
    with pytest.raises(ValueError):
        _shots(v.reshape(-1), src, sp, rp)             # 1-D model
    with pytest.raises(ValueError):
        _shots(v, src, sp, rp[:, :, :1].reshape(3, 5))  # [S][R] is not a receiver list


def test_trace_arrays():
    _check_traces(torch.zeros(3, 40, 5), "obs", 3, 40, 5, torch.device("cpu"))
    for shape in [(3, 40, 4), (3, 39, 5), (2, 40, 5), (40, 5)]:
        with pytest.raises(ValueError):
            _check_traces(torch.zeros(shape), "obs", 3, 40, 5, torch.device("cpu"))


def test_serving_requests_checked():
    import numpy as np

    from paper_1912_08063_amd import serve, workloads as wl
    P = wl.small_2d(nz=20, nx=30, nt=15, nrec=4)
    serve.Server.check_request(serve.Request(0, "forward", 0.0, P))
    g = serve.Request(1, "gradient", 0.0, P, obs=np.zeros((1, 15, 4), np.float32))
    serve.Server.check_request(g)
    serve.Server.check_request(serve.Request(5, "gradient", 0.0, P, obs=g.obs,
                                             ckpt="revolve:3"))
    for bad in (serve.Request(2, "gradient", 0.0, P, obs=np.zeros((1, 14, 4))),
                serve.Request(3, "other", 0.0, P),
                serve.Request(6, "gradient", 0.0, P, obs=g.obs, ckpt="binomial:3"),
                serve.Request(7, "gradient", 0.0, P, obs=g.obs, ckpt="every:")):
        with pytest.raises(ValueError):
            serve.Server.check_request(bad)
    Q = wl.small_2d(nz=20, nx=30, nt=15, nrec=4)
    Q.wavelet = Q.wavelet[:, :10]
    with pytest.raises(ValueError):
        serve.Server.check_request(serve.Request(4, "forward", 0.0, Q))


def test_automatic_checkpoint_policy_fits_its_budget():
    """ckpt="auto:BUDGET" takes every level when they fit, else every-K with the
    K that needs least memory, else binomial checkpointing within the budget;
    each choice's workspace fits the budget."""
    import torch

    from paper_1912_08063_amd import _lib, api
    v = torch.zeros((120, 300))
    cfg = api.Config(dt=1e-3, dx=10.0, order=8, nsponge=20)
    prob = api.make_problem(v, 800, cfg, 4, 50)
    need = lambda spec: _lib.fwi_workspace_bytes(prob, _lib.MODE_GRADIENT, api.parse_ckpt(spec))
    n_all = need("all")
    assert api.choose_ckpt(prob, n_all) == "all"
    assert api.resolve_ckpt("auto:%d" % (n_all + 1), prob, None) == "all"
    mid = api.choose_ckpt(prob, n_all - 1)
    assert mid.startswith("every:")
    k = int(mid.split(":")[1])
    assert abs(k - 40) <= 20          # near sqrt(2 nt) = 40
    assert need(mid) <= n_all - 1
    assert all(need(mid) <= need("every:%d" % j) for j in (5, 20, 80, 200))
    small = need(mid) - 1
    rev = api.choose_ckpt(prob, small)
    assert rev.startswith("revolve:") and need(rev) <= small
    assert api.parse_ckpt(rev).budget_bytes > 0
    assert api.resolve_ckpt("every:50", prob, None) == "every:50"
    # the differentiable forward counts its workspace and its checkpoint buffer
    ck = api.parse_ckpt("all")
    ag_all = (_lib.fwi_workspace_bytes(prob, _lib.MODE_FORWARD_CKPT, ck) +
              _lib.fwi_workspace_bytes(prob, _lib.MODE_CKPT_BUF, ck))
    assert api.choose_ckpt(prob, ag_all, mode="autograd") == "all"
    assert api.choose_ckpt(prob, ag_all - 1, mode="autograd").startswith("every:")
