"""The square root every kernel uses for the objective is a correctly rounded
binary32 sqrt (the oracle's sqrtf): checked bit for bit against numpy's IEEE
float32 sqrt on every non-negative binary32 value, +0 through +inf,
including the subnormals that take the general path."""
import numpy as np
import pytest

import paper_2507_20173_amd as fsb

pytestmark = pytest.mark.gpu
CHUNK = 1 << 27


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch


def test_sqrt_is_correctly_rounded_everywhere(torch_cuda):
    torch = torch_cuda
    end = 0x7F800000 + 1  # +0 .. +inf
    out = torch.empty(CHUNK, dtype=torch.float32, device="cuda")
    bad = 0
    for lo in range(0, end, CHUNK):
        hi = min(lo + CHUNK, end)
        n = hi - lo
        bits = np.arange(lo, hi, dtype=np.uint32)
        x = bits.view(np.float32)
        inp = torch.from_numpy(bits.view(np.int32)).to("cuda").view(torch.float32)
        fsb.fsb_eval_sqrt(inp, out[:n])
        got = out[:n].cpu().numpy().view(np.uint32)
        want = np.sqrt(x).view(np.uint32)
        mism = np.nonzero(got != want)[0]
        if mism.size:
            i = mism[0]
            print(f"[sqrt] {mism.size} mismatches in [{lo:#x}, {hi:#x}), first x bits {bits[i]:#x}: "
                  f"got {got[i]:#x} want {want[i]:#x}", flush=True)
        bad += mism.size
        del inp
    assert bad == 0


def test_sqrt_edge_values(torch_cuda):
    torch = torch_cuda
    vals = np.array([0.0, 2.0**-149, 2.0**-126, 2.0**-96, np.nextafter(np.float32(2.0**-96), np.float32(0)),
                     1.0, 2.0, 20000.0, np.finfo(np.float32).max, np.inf], dtype=np.float32)
    inp = torch.from_numpy(vals).to("cuda")
    out = torch.empty_like(inp)
    fsb.fsb_eval_sqrt(inp, out)
    assert np.array_equal(out.cpu().numpy().view(np.uint32), np.sqrt(vals).view(np.uint32))
