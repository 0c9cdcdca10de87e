"""The stage-handoff probe (a measurement aid): every block writes its slice
and, in modes 1-3, adds 1 to the counter; nothing waits, so every launch ends."""
import numpy as np
import pytest

from gpu_util import device

pytestmark = pytest.mark.gpu


def test_stage_probe_writes_and_counts():
    import torch

    import paper_1709_06999_amd as gal
    from paper_1709_06999_amd import GalarioError

    dev = device()
    blocks = 300
    nb = gal.probe_stage_bytes(blocks)
    assert nb == 256 + blocks * 8192
    ws = torch.zeros(nb, dtype=torch.uint8, device=dev)
    for mode in range(4):
        print(f"stage probe mode {mode}", flush=True)
        gal.probe_stage(mode, blocks, ws)
    torch.cuda.synchronize()
    ctr = int(ws[:4].view(torch.int32).item())
    assert ctr == 3 * blocks
    out = ws[256:].view(torch.float64).cpu().numpy().reshape(blocks, 4, 256)
    expect = np.arange(blocks)[:, None] + np.arange(4)[None, :]
    assert np.array_equal(out, np.broadcast_to(expect[:, :, None], out.shape).astype(np.float64))
    with pytest.raises(GalarioError, match="GAL_ERR_SIZE"):
        gal.probe_stage(4, blocks, ws)
    with pytest.raises(GalarioError, match="GAL_ERR_WORKSPACE"):
        gal.probe_stage(1, blocks + 1, ws)
