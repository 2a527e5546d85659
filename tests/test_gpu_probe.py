"""The tile-march probe (fwi_tile_probe): the forward step's memory pattern
without the stencil writes out = 2 cur + kappa prv at every cell inside the
frame, and nothing else, in every mode and for any chunk length, on a grid
with ragged tiles in x and y and a ragged last chunk in z.

Expected values are plain NumPy arithmetic on the same inputs (the probe is a
diagnostic, not part of the method, so the oracle has nothing to say).  The
kernel computes fma(kappa, prv, 2 cur) in fp32; the NumPy reference in fp64
rounded to fp32, so the two agree to one rounding.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

NZ, NY, NX, M = 37, 21, 70, 4
PITCH = -(-(NX + 2 * M) // 64) * 64
SHAPE = (NZ + 2 * M, NY + 2 * M, PITCH)


def _fields(seed):
    rng = np.random.default_rng(seed)
    return [rng.uniform(-1.0, 1.0, SHAPE).astype(np.float32) for _ in range(3)]


@pytest.mark.parametrize("mode", range(10))
@pytest.mark.parametrize("zc", [0, 1, 5, 36, 37])
def test_tile_probe_writes_the_pointwise_sum_inside_the_frame(mode, zc):
    import torch
    from paper_1912_08063_amd import _lib
    dev = torch.device("cuda:0")
    cur, prv, kap = _fields(1000 + mode)
    sentinel = np.float32(7.25)
    d = [torch.from_numpy(a).to(dev) for a in (cur, prv, kap)]
    out = torch.full(SHAPE, float(sentinel), dtype=torch.float32, device=dev)
    st = torch.cuda.current_stream(dev)
    used = _lib.fwi_tile_probe(d[0].data_ptr(), d[1].data_ptr(), d[2].data_ptr(),
                               out.data_ptr(), NZ, NY, NX, zc, mode, st.cuda_stream)
    torch.cuda.synchronize()
    assert 1 <= used <= NZ and (zc == 0 or used == zc)
    o = out.cpu().numpy()
    inner = (slice(M, M + NZ), slice(M, M + NY), slice(M, M + NX))
    ref = (2.0 * cur.astype(np.float64) + kap.astype(np.float64) * prv.astype(np.float64))
    ref = ref.astype(np.float32)[inner]
    got = o[inner]
    assert np.all(np.abs(got - ref) <= 2 * np.spacing(np.abs(ref)) + 1e-30), mode
    mask = np.ones(SHAPE, dtype=bool)
    mask[inner] = False
    assert np.all(o[mask] == sentinel)
