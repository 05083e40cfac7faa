"""The library's float32 square root against the host's, on every float32 in
[0, 1] (bit patterns 0 .. 0x3F800000: 1,065,353,217 values, subnormals
included), bit for bit.  The ray directions (Sec. 2.2), the coarse SDF
(Sec. 2.1) and the shadow march (Sec. 2.3) take square roots of values in
that range (1 - s of Marsaglia's mapping lies in (0, 1]), and the oracle uses
the host's correctly rounded sqrtf; this is what lets both sides draw
identical rays."""
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

CHUNK = 1 << 27


def test_sqrt_exhaustive_unit_interval():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2210_04449_amd.rtsdf as R
    end = 0x3F800000 + 1
    x = torch.empty(CHUNK, dtype=torch.float32, device="cuda")
    out = torch.empty_like(x)
    mismatches = 0
    for start in range(0, end, CHUNK):
        n = min(CHUNK, end - start)
        bits = torch.arange(start, start + n, dtype=torch.int64, device="cuda").to(torch.int32)
        x[:n] = bits.view(torch.float32)
        R.rtsdf_sqrt(x[:n], out[:n])
        got = out[:n].cpu().numpy()
        want = np.sqrt(np.arange(start, start + n, dtype=np.uint32).view(np.float32))
        bad = got.view(np.uint32) != want.view(np.uint32)
        if bad.any():
            i = int(np.argmax(bad))
            print(f"first mismatch at bits {start + i:#010x}: gpu {got[i]!r} host {want[i]!r}", flush=True)
        mismatches += int(bad.sum())
        print(f"[sqrt] {start + n:#010x} of {end:#010x} checked", flush=True)
        sys.stdout.flush()
    assert mismatches == 0, mismatches
