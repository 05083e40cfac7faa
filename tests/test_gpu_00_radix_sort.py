"""The library's radix sort (the sort of the device rebuild of a hierarchy),
through the C ABI, against numpy's stable argsort: keys and the order of
equal keys (values = input positions) identical, for ragged sizes, heavy
duplication, single-digit and full-width keys.  Runs before the rebuild
tests: the radix-tree builder relies on sorted keys."""
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,bits,hi", [(2, 30, 1 << 30), (5, 8, 3), (4095, 30, 1 << 30), (4097, 30, 64),
                                        (100003, 30, 1 << 30), (1000000, 30, 1 << 30), (262144, 12, 1 << 12),
                                        (300001, 32, 1 << 32), (70000, 16, 1 << 16), (5000, 24, 1)])
def test_sort_pairs_matches_stable_argsort(n, bits, hi):
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2210_04449_amd.rtsdf as R
    print(f"[sort] n={n} bits={bits} hi={hi}", flush=True)
    sys.stdout.flush()
    rng = np.random.default_rng(n + bits)
    keys = rng.integers(0, hi, n, dtype=np.uint64).astype(np.uint32)
    if n > 10:
        keys[: n // 10] = keys[n // 2]  # a long run of one key
    vals = rng.permutation(n).astype(np.int32)
    k = torch.from_numpy(keys.view(np.int32)).cuda()
    v = torch.from_numpy(vals).cuda()
    R.rtsdf_sort_pairs(k, v, bits)
    torch.cuda.synchronize()
    order = np.argsort(keys, kind="stable")
    assert np.array_equal(k.cpu().numpy().view(np.uint32), keys[order])
    assert np.array_equal(v.cpu().numpy(), vals[order])
