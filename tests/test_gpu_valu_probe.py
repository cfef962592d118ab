"""The instrumentation probes.  The VALU ceiling probe: its chains compute
what they claim (checked against closed forms and the oracle's Philox), and
the rates it reports are those of a chip that issues at most a few vector
instructions per SIMD and cycle.  The streaming probe: every element of its
four columns is read and written once per launch, and its rate is below the
memory's peak."""
import numpy as np
import pytest

import paper_2507_20173_amd as fsb
from oracle.oracle import default

pytestmark = pytest.mark.gpu

NOMINAL = 256 * 4 * 16 * 2.4e9  # lane instructions/s, one wave64 issue per SIMD every 4 cycles


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch


def test_fma_chains(torch_cuda):
    torch = torch_cuda
    blocks, iters = 512, 1000
    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    ms, lanes = fsb.fsb_valu_probe(fsb.FSB_PROBE_FMA, blocks, iters, out)
    assert lanes == blocks * 256 * iters * 8 and ms > 0
    # fma(v, 1, 0) keeps every chain at its start value tid + j
    tid = np.arange(blocks * 256) % 256
    assert np.array_equal(out.cpu().numpy(), (8 * tid + 28).astype(np.float32))
    print(f"[probe] fma {lanes / ms / 1e9:.3g} T lane-instructions/s", flush=True)


def test_philox_chains_match_the_oracle(torch_cuda):
    """Each lane feeds Philox4x32-10 its own output `iters` times, from
    counter (lane, j, iters, 0) with key (0x12345678, 0x9ABCDEF0)."""
    torch = torch_cuda
    blocks, iters = 4, 3
    out = torch.empty(blocks * 256, dtype=torch.int32, device="cuda")
    ms, lanes = fsb.fsb_valu_probe(fsb.FSB_PROBE_PHILOX, blocks, iters, out)
    assert lanes == blocks * 256 * iters * 80
    O = default()
    n = blocks * 256
    acc = np.zeros(n, np.uint32)
    keys = np.tile(np.array([0x12345678, 0x9ABCDEF0], np.uint32), (n, 1))
    for j in range(2):
        c = np.stack([np.arange(n, dtype=np.uint32), np.full(n, j, np.uint32),
                      np.full(n, iters, np.uint32), np.zeros(n, np.uint32)], 1)
        for _ in range(iters):
            c = O.philox(c, keys)
        acc ^= c[:, 0] ^ c[:, 1] ^ c[:, 2] ^ c[:, 3]
    assert np.array_equal(out.cpu().numpy().view(np.uint32), acc)


def test_mixed_chains_match_the_oracle(torch_cuda):
    """One Philox call per round from counter (lane, 7, iters, 0), beside fma
    chains that keep their start values; the two folded into one word."""
    torch = torch_cuda
    blocks, iters = 2, 5
    out = torch.empty(blocks * 256, dtype=torch.int32, device="cuda")
    ms, lanes = fsb.fsb_valu_probe(fsb.FSB_PROBE_MIXED, blocks, iters, out)
    assert lanes == blocks * 256 * iters * 80
    O = default()
    n = blocks * 256
    keys = np.tile(np.array([0x12345678, 0x9ABCDEF0], np.uint32), (n, 1))
    c = np.stack([np.arange(n, dtype=np.uint32), np.full(n, 7, np.uint32),
                  np.full(n, iters, np.uint32), np.zeros(n, np.uint32)], 1)
    for _ in range(iters):
        c = O.philox(c, keys)
    tid = np.arange(n) % 256
    acc = (8 * tid + 28).astype(np.float32).view(np.uint32)
    want = c[:, 0] ^ c[:, 1] ^ c[:, 2] ^ c[:, 3] ^ acc
    assert np.array_equal(out.cpu().numpy().view(np.uint32), want)


@pytest.mark.parametrize("kind", [0, 1, 2], ids=["fma", "philox", "mixed"])
def test_rates_are_plausible(torch_cuda, kind):
    """From one wave per SIMD to eight: the rate rises with the waves and stays
    below twice the nominal issue rate (no lane can retire two instructions
    per cycle without dual issue)."""
    torch = torch_cuda
    rates = []
    for waves in (1, 2, 4, 8):
        blocks = 256 * waves
        out = torch.empty(blocks * 256, dtype=torch.int32, device="cuda")
        fsb.fsb_valu_probe(kind, blocks, 64, out)  # warm-up
        ms, lanes = fsb.fsb_valu_probe(kind, blocks, 2048 if kind == 0 else 256, out)
        rates.append(lanes / (ms / 1e3))
        print(f"[probe] kind {kind} waves/SIMD {waves}: {rates[-1] / 1e12:.2f} T", flush=True)
    assert rates[-1] >= rates[0] * 0.9
    assert all(0 < r < 2 * NOMINAL for r in rates)


def test_probe_rejects_bad_arguments(torch_cuda):
    torch = torch_cuda
    out = torch.empty(256, dtype=torch.float32, device="cuda")
    for kind, blocks, iters in ((3, 1, 1), (0, 0, 1), (0, 1, 0)):
        with pytest.raises(fsb.FsbError):
            fsb.fsb_valu_probe(kind, blocks, iters, out)


@pytest.mark.parametrize("n,streamed", [(4096, False), ((1 << 22) + 4, True), (1 << 24, False)])
def test_sweep_probe_touches_every_element_once(torch_cuda, n, streamed):
    torch = torch_cuda
    cols = [torch.full((n,), float(k), dtype=torch.float32, device="cuda") for k in range(4)]
    ms = fsb.fsb_sweep_probe(cols, 0, streamed)
    ms += fsb.fsb_sweep_probe(cols, 0, streamed)
    for k, c in enumerate(cols):
        assert torch.equal(c, torch.full_like(c, k + 2.0)), k
    rate = 2 * 32 * n / (ms / 1e3) / 1e9
    print(f"[probe] sweep n={n} streamed={streamed}: {rate:.0f} GB/s", flush=True)
    assert ms > 0 and (n < 1 << 20 or rate < 2 * 8000)
